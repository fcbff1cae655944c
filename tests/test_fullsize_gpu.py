"""Parity at the full workload sizes, in the launch configuration the
benchmark times (default block 256, 4 points per lane).

* ACOPF-shaped, 10,000 buses: every output compared in full with the oracle.
* PDE control, n = 1000 (2e6 variables): structure in full, obj/grad/cons in
  full, Jacobian and Hessian values at 4,000 sampled data points per pattern
  (the oracle evaluates just those points), products through properties.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from exa_modeling.generators import acopf, goddard, pde
from oracle import OracleModel
from parity_util import abs_oracle, assert_close, column_scale, dev, host
from test_parity_gpu import check_all

pytestmark = pytest.mark.gpu


def test_acopf_10k_all_callbacks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    check_all(acopf(10000, 1), tag="acopf10k: ")


def test_pde_1000_sampled():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_16265_amd import ExaModel
    w = pde(1000, 3)
    em = ExaModel(w.model)
    o = OracleModel(w.model)
    x, y = w.x, w.y
    X, Y = dev(x), dev(y)
    for g, r in zip(em.jac_structure(), o.jac_structure()):
        assert np.array_equal(g, r)
    for g, r in zip(em.hess_structure(), o.hess_structure()):
        assert np.array_equal(g, r)
    assert_close("obj", host(em.obj(X))[0], o.obj(x),
                 float(sum(np.sum(np.abs(o.pattern_values(i, x))) for i in (0, 1))))
    assert_close("cons", host(em.cons(X)), o.cons(x), np.abs(o.cons(x)) + 1.0)
    J = host(em.jac_coord(X))
    H = host(em.hess_coord(X, Y, 1.0))
    rng = np.random.default_rng(9)
    for i, P in enumerate(o.pats):
        ks = np.unique(np.concatenate([rng.integers(0, P.ndata, 4000), [0, P.ndata - 1]]))
        if P.kind != "obj" and P.vslots:
            st = len(P.vslots)
            ref = o.jac_block(i, ks, x)
            got = J[P.o1 + ks[:, None] * st + np.arange(st)]
            assert_close(f"jac[{i}]", got, ref, np.abs(ref).max(axis=0))
        if P.hslots:
            st = len(P.hslots)
            ref = o.hess_block(i, ks, x, y, 1.0)
            got = H[P.o2 + ks[:, None] * st + np.arange(st)]
            assert_close(f"hess[{i}]", got, ref, np.abs(ref).max(axis=0))
    # products through their definition on the full vectors: J v from COO
    v = rng.standard_normal(o.nvar)
    import scipy.sparse as sp
    rj, cj = o.jac_structure()
    # absolute values are taken entry by entry, before duplicates are summed
    def sym(vals, r, c):
        L = sp.coo_matrix((vals, (r, c)), shape=(o.nvar, o.nvar)).tocsr()
        return L + L.T - sp.diags(L.diagonal())
    Jm = sp.coo_matrix((J, (rj, cj)), shape=(o.ncon, o.nvar)).tocsr()
    Ja = sp.coo_matrix((np.abs(J), (rj, cj)), shape=(o.ncon, o.nvar)).tocsr()
    assert_close("jprod", host(em.jprod(X, dev(v))), Jm @ v, Ja @ np.abs(v))
    rh, ch = o.hess_structure()
    assert_close("hprod", host(em.hprod(X, Y, 1.0, dev(v))), sym(H, rh, ch) @ v,
                 sym(np.abs(H), rh, ch) @ np.abs(v))


def test_goddard_large_reductions():
    """Goddard rocket with 300,000 steps: the step variable's Jacobian column
    holds 900,000 entries and every other column at most 16, so J^T w, H v
    and the Lagrangian gradient take the large-map reduction (one lane per
    short segment, parts for the long one).  Checked against scipy's COO
    products of the device's own COO values (the values themselves are
    checked against the oracle at smaller sizes) and bit for bit across
    exa_eval, the single callbacks and repeated calls."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import scipy.sparse as sp
    from paper_2608_16265_amd import ExaModel
    w = goddard(300000, 0)
    em = ExaModel(w.model)
    rng = np.random.default_rng(9)
    X, Y = dev(w.x), dev(w.y)
    v, wv = rng.standard_normal(em.nvar), rng.standard_normal(em.ncon)
    V, W = dev(v), dev(wv)
    rj, cj = em.jac_structure()
    rh, ch = em.hess_structure()
    jv, hv = host(em.jac_coord(X)), host(em.hess_coord(X, Y, 1.0))
    J = sp.coo_matrix((jv, (rj, cj)), shape=(em.ncon, em.nvar)).tocsr()
    Ja = sp.coo_matrix((np.abs(jv), (rj, cj)), shape=(em.ncon, em.nvar)).tocsr()
    L = sp.coo_matrix((hv, (rh, ch)), shape=(em.nvar, em.nvar)).tocsr()
    La = sp.coo_matrix((np.abs(hv), (rh, ch)), shape=(em.nvar, em.nvar)).tocsr()
    H = L + L.T - sp.diags(L.diagonal())
    Ha = La + La.T - sp.diags(La.diagonal())
    jt = host(em.jtprod(X, W))
    assert_close("jtprod", jt, J.T @ wv, Ja.T @ np.abs(wv), rtol=1e-13)
    assert_close("hprod", host(em.hprod(X, Y, 1.0, V)), H @ v, Ha @ np.abs(v), rtol=1e-13)
    g = host(em.grad(X))
    lg = host(em.lag_grad(X, Y, 1.0))
    assert np.array_equal(lg, host(dev(g).mul_(1.0).add_(em.jtprod(X, Y))))
    out = torch.empty(em.nvar, dtype=torch.float64, device="cuda:0")
    em.evaluate(X, Y, 1.0, V, W, jtw=out)
    assert np.array_equal(host(out), jt)
    for _ in range(3):
        assert np.array_equal(host(em.jtprod(X, W)), jt)


ALL = ("f", "g", "c", "jac", "hess", "jv", "jtw", "hv")


def _eval_tuned(em, X, Y, V, W):
    """Every callback through one exa_eval call under the tuned schedule,
    as the benchmark's step runs it (twice: tuning happens at the first)."""
    e = lambda n: torch.empty(n, dtype=torch.float64, device="cuda:0")  # noqa: E731
    outs = dict(f=e(1), g=e(em.nvar), c=e(em.ncon), jac=e(em.nnzj), hess=e(em.nnzh), jv=e(em.ncon),
                jtw=e(em.nvar), hv=e(em.nvar))
    step = em.bind(X, Y, 1.0, V, W, **outs)
    step()
    for t in outs.values():
        t.fill_(float("nan"))
    step()
    torch.cuda.synchronize()
    return {k: host(t) for k, t in outs.items()}


def _worst(got, ref, scale):
    got, ref = np.asarray(got, dtype=np.longdouble), np.asarray(ref, dtype=np.longdouble)
    tol = 1e-12 * np.maximum(np.abs(ref), np.asarray(scale, dtype=np.longdouble))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(tol > 0, np.abs(got - ref) / tol, np.where(got == ref, 0.0, np.inf))
    return float(np.max(r)) if r.size else 0.0


def test_acopf_10k_eval_tuned_matches_oracle_with_error_report():
    """The benchmark's 10k step (exa_eval of every callback, autotuned)
    against the oracle in full, and the true error of both against the
    oracle evaluated in x87 extended precision: worst |err| / tol per
    callback, printed (tol = 1e-12 max(|ref|, column scale))."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_16265_amd import ExaModel
    w = acopf(10000, 1)
    em = ExaModel(w.model, autotune=True)
    o = OracleModel(w.model)
    rng = np.random.default_rng(0)
    v, wv = rng.standard_normal(o.nvar), rng.standard_normal(o.ncon)
    got = _eval_tuned(em, dev(w.x), dev(w.y), dev(v), dev(wv))
    a = abs_oracle(o, w.x, w.y, 1.0, v, wv)
    ld = np.longdouble
    refs = {
        "f": (lambda d: np.array([o.obj(w.x, dtype=d)]), np.array([a["obj"]])),
        "g": (lambda d: o.grad(w.x, dtype=d), a["grad"]),
        "c": (lambda d: o.cons(w.x, dtype=d), a["cons"]),
        "jac": (lambda d: o.jac_coord(w.x, dtype=d), None),
        "hess": (lambda d: o.hess_coord(w.x, w.y, 1.0, dtype=d), None),
        "jv": (lambda d: o.jprod(w.x, v, dtype=d), a["jprod"]),
        "jtw": (lambda d: o.jtprod(w.x, wv, dtype=d), a["jtprod"]),
        "hv": (lambda d: o.hprod(w.x, w.y, 1.0, v, dtype=d), a["hprod"]),
    }
    report = {}
    for k, (f, scale) in refs.items():
        r64 = f(np.float64)
        if k in ("jac", "hess"):
            scale = column_scale(o, r64, 1 if k == "jac" else 2)
        assert_close("acopf10k eval " + k, got[k], r64, scale)
        rld = f(ld)
        report[k] = (_worst(got[k], rld, scale), _worst(r64, rld, scale))
    for k, (g_, o_) in report.items():
        print(f"acopf10k {k}: worst |gpu - ref_ld| / tol = {g_:.3e}; worst |oracle64 - ref_ld| / tol = {o_:.3e}")
    assert all(g_ <= 1.0 for g_, _ in report.values())


def test_pde_1000_eval_tuned_sampled():
    """The benchmark's PDE step (exa_eval of every callback, autotuned) at
    n = 1000: objective, gradient and constraints in full against the
    oracle, Jacobian and Hessian at sampled data points, products through
    their definition on the full COO values, and every output bit for bit
    equal to the single callbacks."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import scipy.sparse as sp
    from paper_2608_16265_amd import ExaModel
    w = pde(1000, 3)
    em = ExaModel(w.model, autotune=True)
    o = OracleModel(w.model)
    x, y = w.x, w.y
    rng = np.random.default_rng(4)
    v, wv = rng.standard_normal(o.nvar), rng.standard_normal(o.ncon)
    X, Y, V, W = dev(x), dev(y), dev(v), dev(wv)
    got = _eval_tuned(em, X, Y, V, W)
    single = dict(f=em.obj(X), g=em.grad(X), c=em.cons(X), jac=em.jac_coord(X), hess=em.hess_coord(X, Y, 1.0),
                  jv=em.jprod(X, V), jtw=em.jtprod(X, W), hv=em.hprod(X, Y, 1.0, V))
    for k in ALL:
        assert np.array_equal(got[k], host(single[k])), f"pde eval {k} differs from its callback"
    a_obj = float(sum(np.sum(np.abs(o.pattern_values(i, x))) for i in (0, 1)))
    assert_close("pde obj", got["f"][0], o.obj(x), a_obj)
    gr = o.grad(x)
    assert_close("pde grad", got["g"], gr, np.abs(gr))
    assert_close("pde cons", got["c"], o.cons(x), np.abs(o.cons(x)) + 1.0)
    J, H = got["jac"], got["hess"]
    for i, P in enumerate(o.pats):
        ks = np.unique(np.concatenate([rng.integers(0, P.ndata, 4000), [0, P.ndata - 1]]))
        if P.kind != "obj" and P.vslots:
            st = len(P.vslots)
            ref = o.jac_block(i, ks, x)
            assert_close(f"pde jac[{i}]", J[P.o1 + ks[:, None] * st + np.arange(st)], ref, np.abs(ref).max(axis=0))
        if P.hslots:
            st = len(P.hslots)
            ref = o.hess_block(i, ks, x, y, 1.0)
            assert_close(f"pde hess[{i}]", H[P.o2 + ks[:, None] * st + np.arange(st)], ref, np.abs(ref).max(axis=0))
    rj, cj = o.jac_structure()
    rh, ch = o.hess_structure()
    Jm = sp.coo_matrix((J, (rj, cj)), shape=(o.ncon, o.nvar)).tocsr()
    Ja = sp.coo_matrix((np.abs(J), (rj, cj)), shape=(o.ncon, o.nvar)).tocsr()

    def sym(vals):
        L = sp.coo_matrix((vals, (rh, ch)), shape=(o.nvar, o.nvar)).tocsr()
        return L + L.T - sp.diags(L.diagonal())
    assert_close("pde jprod", got["jv"], Jm @ v, Ja @ np.abs(v))
    assert_close("pde jtprod", got["jtw"], Jm.T @ wv, Ja.T @ np.abs(wv))
    assert_close("pde hprod", got["hv"], sym(H) @ v, sym(np.abs(H)) @ np.abs(v))
