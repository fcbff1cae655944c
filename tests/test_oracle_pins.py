"""The CPU oracle against values fixed by the paper and by mathematics."""
import json
import math
import os

import numpy as np
import pytest

from exa_modeling import DataSet, Model, cos, sin, exp
from exa_modeling.generators import Workload, acopf, goddard, kernel_sweep, pde, rosenbrock, two_stage
from oracle import OracleModel, rules
from oracle_checks import check_aug_offset, check_coverage, check_first_order, check_second_order

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


# ----------------------------------------------------------------- paper values
def test_rosenbrock_node_values():
    g = GOLD["rosenbrock_node_eval"]
    w = rosenbrock(3)
    o = OracleModel(w.model)
    vals = o.pattern_values(0, np.array(g["x"]))
    # data point i (1-based) is entry i-2 of the 0-based range 1..N-1
    assert [vals[p - 2] for p in g["points"]] == g["values"]


def test_product_value_and_gradient():
    g = GOLD["product_adjoint"]
    m = Model()
    x = m.add_var(2)
    m.add_obj(x[0] ** 2 * x[1], DataSet(1, k=np.zeros(1, dtype=np.int32)))
    o = OracleModel(m)
    xv = np.array(g["x"])
    assert o.obj(xv) == g["value"]
    assert list(o.grad(xv)) == g["gradient"]


def test_rosenbrock_gradient_worked_example():
    g = GOLD["rosenbrock_gradient"]
    w = rosenbrock(2)
    o = OracleModel(w.model)
    assert list(o.grad(np.array(g["x"]))) == g["gradient"]


def test_rosenbrock_probe_and_compressors():
    g = GOLD["rosenbrock_probe"]
    o = OracleModel(rosenbrock(5).model)
    pr = o.probe(0)
    assert [k[2] for k in pr["raw1"]] == g["raw1_shifts"]
    assert pr["comp1"] == g["comp1"] and pr["o1step"] == g["o1step"]
    assert pr["comp2"] == g["comp2"] and pr["o2step"] == g["o2step"]
    slots = o.pats[0].hslots
    assert sum(a == b for a, b in slots) == g["n_diagonal"]
    assert sum(a != b for a, b in slots) == g["n_offdiagonal"]


def test_write_positions():
    g = GOLD["write_position"]
    # two objective terms ahead of Rosenbrock occupy Jacobian-free space; use a
    # constraint pattern so the o1 offset is exercised: a 1-entry pattern first.
    m = Model()
    x = m.add_var(4)
    d1 = DataSet(2, k=np.arange(2))
    m.add_con(x[d1.k], d1)                     # 2 entries -> o1 of the next = 2
    d = DataSet(3, i=np.arange(1, 4))
    i = d.i
    m.add_con(100 * (x[i - 1] ** 2 - x[i]) ** 2 + (x[i - 1] - 1) ** 2, d)
    o = OracleModel(m)
    P = o.pats[1]
    assert P.o1 == g["o1"] and len(P.vslots) == g["o1step"] and P.comp1 == g["comp1"]
    rows, cols = o.jac_structure()
    for k, want in ((1, g["positions_k1"]), (2, g["positions_k2"])):
        got = [P.o1 + (k - 1) * len(P.vslots) + c for c in P.comp1]
        assert got == want
        # the entries at those (1-based) positions are the rows of point k
        assert all(rows[p - 1] == 2 + (k - 1) for p in got)


def test_simplification_table():
    for op, a, b, want in GOLD["simplification_table"]["rules"]:
        def leaf(v):
            if v == "x":
                return rules.T("var", col=None, off=0)
            return rules.T("const", value=float(v))
        t = rules.simplify(rules.T(op, (leaf(a), leaf(b))))
        if want == "x":
            assert t.op == "var"
        elif want == "abs2(x)":
            assert t.op == "abs2" and t.args[0].op == "var"
        elif want == "inv(x)":
            assert t.op == "inv" and t.args[0].op == "var"
        else:
            assert t.op == "const" and t.value == float(want)
    # commutative forms and non-rules
    v = rules.T("var", off=0)
    c0, c1 = rules.T("const", value=0.0), rules.T("const", value=1.0)
    assert rules.simplify(rules.T("add", (c0, v))).op == "var"
    assert rules.simplify(rules.T("mul", (c1, v))).op == "var"
    assert rules.simplify(rules.T("mul", (v, c0))).op == "const"
    assert rules.simplify(rules.T("sub", (v, c0))).op == "sub"
    assert rules.simplify(rules.T("pow", (v, rules.T("const", value=3.0)))).op == "pow"


# -------------------------------------------------------------- closed forms
def test_rosenbrock_hessian_closed_form():
    o = OracleModel(rosenbrock(2).model)
    x = np.array([2.0, 3.0])
    H = o.hess_matrix(x, np.zeros(0), 1.0).toarray()
    x1, x2 = x
    assert H[0, 0] == 1200 * x1 ** 2 - 400 * x2 + 2 == 3602
    assert H[1, 0] == H[0, 1] == -400 * x1 == -800
    assert H[1, 1] == 200


def test_acopf_flow_partials_closed_form():
    w = acopf(30, 0)
    o = OracleModel(w.model)
    md = w.meta
    nb, nl = md["nb"], md["nl"]
    off = md["offsets"]
    x = w.x
    J = o.jac_matrix(x).tocsr()
    br = w.model.patterns[1].data
    g, b = br.fcols["g"], br.fcols["b"]
    for l in range(nl):
        f, t = int(br.icols["f"][l]), int(br.icols["t"][l])
        vf, vt = x[off["vm"] + f], x[off["vm"] + t]
        th = x[off["va"] + f] - x[off["va"] + t]
        row = l  # C_pf is the first constraint block
        want = {
            off["p"] + l: 1.0,
            off["vm"] + f: -(2 * g[l] * vf - vt * (g[l] * math.cos(th) + b[l] * math.sin(th))),
            off["vm"] + t: vf * (g[l] * math.cos(th) + b[l] * math.sin(th)),
            off["va"] + f: vf * vt * (-g[l] * math.sin(th) + b[l] * math.cos(th)),
            off["va"] + t: -vf * vt * (-g[l] * math.sin(th) + b[l] * math.cos(th)),
        }
        for col, val in want.items():
            assert abs(J[row, col] - val) <= 1e-13 * max(1.0, abs(val))


def test_quadratic_hessians_exact():
    w = acopf(30, 0)
    o = OracleModel(w.model)
    vals = o.hess_coord(w.x, w.y, 2.5)
    P0 = o.pats[0]
    c2 = w.model.theta[w.meta["theta_offsets"]["c2"]:][:w.meta["ng"]]
    assert np.array_equal(vals[P0.o2:P0.o2 + P0.ndata], 2 * c2 * 2.5)
    Tf = o.pats[11]
    rows = Tf.o0 + np.arange(Tf.ndata)
    blk = vals[Tf.o2:Tf.o2 + 2 * Tf.ndata].reshape(-1, 2)
    assert np.array_equal(blk[:, 0], 2 * w.y[rows]) and np.array_equal(blk[:, 1], 2 * w.y[rows])


def test_pde_closed_forms():
    w = pde(6, 3)
    o = OracleModel(w.model)
    n, h = w.meta["n"], w.meta["h"]
    ih2 = (n - 1) ** 2
    x, y = w.x, w.y
    vals = o.jac_coord(x)
    P = o.pats[2]
    inter = w.meta["interior"]
    blk = vals[P.o1:].reshape(-1, 6)
    uc = x[inter]
    assert np.allclose(blk[:, 0], 4 * ih2 + np.exp(uc), rtol=1e-15, atol=0)
    assert np.all(blk[:, 1:5] == -ih2) and np.all(blk[:, 5] == -1.0)
    hv = o.hess_coord(x, y, 1.5)
    N = n * n
    assert np.all(hv[:N] == 1.5) and np.all(hv[N:2 * N] == 2e-4 * 1.5)
    assert np.allclose(hv[2 * N:], y * np.exp(uc), rtol=1e-15, atol=0)


def test_dims_formulae():
    for nb, seed in ((30, 0), (97, 5)):
        w = acopf(nb, seed)
        o = OracleModel(w.model)
        nl, ng = w.meta["nl"], w.meta["ng"]
        assert o.dims() == (2 * nb + 2 * ng + 4 * nl, 6 * nl + 2 * nb, 28 * nl + 2 * ng, 40 * nl + ng)


# ---------------------------------------------------- complex step / FD / coverage
@pytest.mark.parametrize("name", ["acopf30", "pde8", "rosen5", "goddard6", "sweep16", "twostage"])
def test_first_order_vs_complex_step(name):
    wl = {"acopf30": lambda: acopf(30, 0), "pde8": lambda: pde(8, 3),
          "rosen5": lambda: rosenbrock(5, 1), "goddard6": lambda: goddard(6, 2),
          "sweep16": lambda: kernel_sweep(16, 32, 1), "twostage": lambda: two_stage(3, 2, 4, 1)}[name]()
    assert check_first_order(wl) < 1e-13


@pytest.mark.parametrize("name", ["acopf30", "pde8", "rosen5", "goddard6", "sweep16", "twostage"])
def test_hessian_vs_fd_of_gradient(name):
    wl = {"acopf30": lambda: acopf(30, 0), "pde8": lambda: pde(8, 3),
          "rosen5": lambda: rosenbrock(5, 1), "goddard6": lambda: goddard(6, 2),
          "sweep16": lambda: kernel_sweep(16, 32, 1), "twostage": lambda: two_stage(3, 2, 4, 1)}[name]()
    assert check_second_order(wl) < 1e-6


@pytest.mark.parametrize("name", ["acopf30", "pde8", "rosen5", "ops", "goddard6", "sweep16", "twostage"])
def test_structure_covers_local_hessians(name):
    wl = {"acopf30": lambda: acopf(30, 0), "pde8": lambda: pde(8, 3),
          "rosen5": lambda: rosenbrock(5, 1), "ops": lambda: op_zoo(), "goddard6": lambda: goddard(6, 2),
          "sweep16": lambda: kernel_sweep(16, 32, 1), "twostage": lambda: two_stage(3, 2, 4, 1)}[name]()
    assert check_coverage(wl) == 0.0


def op_zoo(seed=7):
    """Every operator of the vocabulary, in a few small patterns."""
    from exa_modeling import ir
    rng = np.random.default_rng(seed)
    m = Model("zoo")
    x = m.add_var(6)
    th = m.add_par(rng.uniform(0.5, 1.5, 3))
    d = DataSet(5, i=np.arange(5) % 3, j=(np.arange(5) + 1) % 3, c=rng.uniform(0.5, 2.0, 5))
    a, b, c = x[d.i], x[d.j + 3], x[d.i + 3]
    m.add_obj(ir.exp(a) * ir.sin(b) + ir.log(c) / (a + 3) + ir.sqrt(c) * th[d.i], d)
    m.add_con(ir.tan(a / 4) + ir.atan(b) * ir.cos(c) - ir.inv(c) + a ** 3, d)
    m.add_con(ir.sinh(a) * ir.cosh(b) + ir.tanh(c) ** 2 + ir.log1p(c) - ir.expm1(a) / d.c, d)
    m.add_con(c ** b + 2.0 ** a + (-a) * th[d.j] + c ** d.c, d)
    xv = np.concatenate([rng.uniform(-1, 1, 3), rng.uniform(0.5, 2.0, 3)])
    return Workload(m, xv, rng.standard_normal(m.ncon), 0.7)


def test_op_zoo_first_and_second_order():
    wl = op_zoo()
    assert check_first_order(wl) < 1e-13
    assert check_second_order(wl) < 1e-6


# ------------------------------------------------------------------- aliasing
def test_aliased_references_sum_to_true_hessian():
    """x[d.i] * x[d.j] with d.i == d.j at some points: duplicates must sum to
    the true Hessian (the cross entry carries twice the mixed derivative)."""
    m = Model()
    x = m.add_var(3)
    d = DataSet(3, i=np.array([0, 1, 2]), j=np.array([0, 2, 2]))
    m.add_obj(exp(x[d.i] * x[d.j]), d)
    o = OracleModel(m)
    xv = np.array([0.3, -0.2, 0.5])
    H = o.hess_matrix(xv, np.zeros(0), 1.0).toarray()
    Hfd = np.zeros((3, 3))
    # closed form: sum over points of exp(xi xj) terms
    for i, j in zip([0, 1, 2], [0, 2, 2]):
        xi, xj = xv[i], xv[j]
        if i == j:
            Hfd[i, i] += (2 + 4 * xi * xi) * math.exp(xi * xi)
        else:
            e = math.exp(xi * xj)
            Hfd[i, i] += xj * xj * e
            Hfd[j, j] += xi * xi * e
            Hfd[i, j] += (1 + xi * xj) * e
            Hfd[j, i] += (1 + xi * xj) * e
    assert np.allclose(H, Hfd, rtol=1e-14, atol=0)


# ------------------------------------------------------------------- adjoint
def test_adjoint_closed_forms_acopf():
    w = acopf(30, 0)
    o = OracleModel(w.model)
    rng = np.random.default_rng(11)
    wv = rng.standard_normal(o.nvar)
    sig = 1.3
    tb = o.adjoint_theta(w.x, w.y, sig, wv)
    to = w.meta["theta_offsets"]
    nb, ng = w.meta["nb"], w.meta["ng"]
    pg = w.x[w.meta["offsets"]["pg"]:][:ng]
    wpg = wv[w.meta["offsets"]["pg"]:][:ng]
    assert np.all(tb[to["pd"]:to["pd"] + nb] == 0.0)
    assert np.all(tb[to["qd"]:to["qd"] + nb] == 0.0)
    assert np.array_equal(tb[to["c1"]:to["c1"] + ng], sig * wpg)
    assert np.allclose(tb[to["c2"]:to["c2"] + ng], 2 * sig * pg * wpg, rtol=1e-15, atol=0)


def test_adjoint_vs_fd_with_branch_parameters():
    """g and b moved into theta make the adjoint non-degenerate; check it by
    central differences (h = 1e-6) of w . grad_x L(theta)."""
    w = acopf(30, 0, gb_in_theta=True)
    o = OracleModel(w.model)
    rng = np.random.default_rng(5)
    wv = rng.standard_normal(o.nvar)
    th = w.model.theta
    tb = o.adjoint_theta(w.x, w.y, 1.0, wv)
    h = 1e-6
    fd = np.zeros_like(th)
    for t in range(th.size):
        tp, tm = th.copy(), th.copy()
        tp[t] += h
        tm[t] -= h
        fd[t] = (wv @ o.grad_lagrangian(w.x, w.y, 1.0, tp) - wv @ o.grad_lagrangian(w.x, w.y, 1.0, tm)) / (2 * h)
    assert np.max(np.abs(tb - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))
    assert np.max(np.abs(tb[-2 * w.meta["nl"]:])) > 1.0   # the g, b part is not zero


def test_products_match_dense():
    w = acopf(30, 0)
    o = OracleModel(w.model)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(o.nvar)
    J = o.jac_matrix(w.x).toarray()
    H = o.hess_matrix(w.x, w.y, 0.8).toarray()
    assert np.allclose(o.jprod(w.x, v), J @ v, rtol=1e-14, atol=1e-12)
    assert np.allclose(o.hprod(w.x, w.y, 0.8, v), H @ v, rtol=1e-14, atol=1e-12)
    assert np.allclose(H, H.T)


# ------------------------------------------------- augmentation row offsets
def aug_offset_case(seed=12):
    """Augmentations whose row is an index column plus a nonzero offset
    (eq. simd:con, Sec. 3.3.2), added to a base block that is not the first,
    so that the target block's first row, the index column and the offset
    all enter the row: c_k sin(x_j) x_m into row bus_k + 2 of block B and
    exp(x_j) into row bus_k - 1 of block B."""
    rng = np.random.default_rng(seed)
    m = Model("augoff")
    n = 12
    x = m.add_var(n)
    a = DataSet(3, i=np.arange(3))
    m.add_con(x[a.i] * x[a.i + 1], a)               # block A: rows 0..2
    r = DataSet(8, r=np.arange(8))
    blk = m.add_con(x[r.r] ** 2, r)                  # block B: rows 3..10
    K = 10
    j = rng.integers(0, n, K)
    mm = (j + 1 + rng.integers(0, n - 1, K)) % n    # never equal to j
    d1 = dict(bus=rng.integers(0, 6, K), j=j, m=mm, c=rng.uniform(0.5, 2.0, K))
    d = DataSet(K, **d1)
    m.add_con_aug(blk, d.bus + 2, d.c * sin(x[d.j]) * x[d.m], d)
    d2 = dict(bus=rng.integers(1, 9, 6), j=rng.integers(0, n, 6))
    e = DataSet(6, **d2)
    m.add_con_aug(blk, e.bus - 1, exp(x[e.j]), e)
    xv = rng.uniform(-1.0, 1.0, n)
    return Workload(m, xv, rng.standard_normal(m.ncon), 0.9, dict(aug1=d1, aug2=d2))


def test_aug_row_offset_closed_form():
    wl = aug_offset_case()
    assert [p.row_off for p in wl.model.patterns[2:]] == [2, -1]
    assert check_aug_offset(wl) < 1e-15


def test_aug_row_offset_first_and_second_order():
    wl = aug_offset_case()
    assert check_first_order(wl) < 1e-13
    assert check_second_order(wl) < 1e-6


# --------------------------------------- sampled blocks = the full arrays
@pytest.mark.parametrize("name", ["acopf30", "pde8", "alias", "augoff", "goddard6"])
def test_blocks_equal_coord_slices(name):
    """jac_block / hess_block (used to check sampled points of large
    models) give, at every data point, exactly the entries of jac_coord /
    hess_coord, which the closed forms, complex step and FD pin."""
    def alias():
        m = Model()
        x = m.add_var(3)
        d = DataSet(3, i=np.array([0, 1, 2]), j=np.array([0, 2, 2]))
        m.add_obj(exp(x[d.i] * x[d.j]), d)
        m.add_con(sin(x[d.i]) * x[d.j], d)
        return Workload(m, np.array([0.3, -0.2, 0.5]), np.array([0.7, -1.1, 0.4]), 1.3)
    wl = {"acopf30": lambda: acopf(30, 0), "pde8": lambda: pde(8, 3), "alias": alias,
          "augoff": aug_offset_case, "goddard6": lambda: goddard(6, 2)}[name]()
    o = OracleModel(wl.model)
    J = o.jac_coord(wl.x)
    H = o.hess_coord(wl.x, wl.y, wl.sigma)
    for i, P in enumerate(o.pats):
        ks = np.arange(P.ndata)[::-1]       # any order of points
        if P.kind != "obj" and P.vslots:
            st = len(P.vslots)
            blk = o.jac_block(i, ks, wl.x)
            assert np.array_equal(blk, J[P.o1:P.o1 + P.ndata * st].reshape(P.ndata, st)[ks])
        if P.hslots:
            st = len(P.hslots)
            blk = o.hess_block(i, ks, wl.x, wl.y, wl.sigma)
            assert np.array_equal(blk, H[P.o2:P.o2 + P.ndata * st].reshape(P.ndata, st)[ks])


# --------------------------------------------- extended-precision reference
def test_longdouble_reference_agrees():
    """The oracle evaluated in x87 extended precision (64-bit significand)
    is the reference for reporting true errors; in float64 it must agree
    with it to the parity tolerance on the 30-bus model."""
    from parity_util import column_scale
    assert np.finfo(np.longdouble).nmant >= 63
    wl = acopf(30, 0)
    o = OracleModel(wl.model)
    ld = np.longdouble
    for f, order in ((lambda d: o.jac_coord(wl.x, dtype=d), 1),
                     (lambda d: o.hess_coord(wl.x, wl.y, 1.0, dtype=d), 2)):
        a, b = f(np.float64), f(ld)
        assert b.dtype == ld
        sc = column_scale(o, a, order)
        err = np.abs(a.astype(ld) - b)
        assert np.all(err <= 1e-12 * np.maximum(np.abs(b), sc))
        assert np.any(err > 0)            # the two precisions really differ
