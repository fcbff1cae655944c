"""Batched evaluation: every instance's outputs of every callback are
bit-identical to the plain per-instance calls, for uneven instance sizes,
every schedule, graph replays and eager launches; against the oracle on
instances of the 256-instance workload."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from exa_modeling.generators import acopf, acopf_batch, acopf_batch_instance, goddard, two_stage
from oracle import OracleModel
from parity_util import abs_oracle, adjoint_scale, assert_close, column_scale, dev, host

pytestmark = pytest.mark.gpu

ALL8 = dict(f="B", g="x", c="y", jac="jac", hess="hess", jv="y", jtw="x", hv="x")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(b, wls, seed=3):
    rng = np.random.default_rng(seed)
    X = b.concat([w.x for w in wls])
    Y = b.concat([w.y for w in wls])
    V = dev(rng.standard_normal(b.total("x")))
    W = dev(rng.standard_normal(b.total("y")))
    WX = dev(rng.standard_normal(b.total("x")))
    return X, Y, V, W, WX


def _nan(b, kind):
    return torch.full((b.total(kind),), np.nan, dtype=torch.float64, device="cuda:0")


def _check_against_plain(b, ems, X, Y, V, W, WX, sigma, outs, lag=None, tbar=None, tag=""):
    """Each instance's slice of every output equals its own callback."""
    torch.cuda.synchronize()
    for i, e in enumerate(ems):
        sx, sy = b.slice("x", i), b.slice("y", i)
        x, y, v, w, wx = X[sx].clone(), Y[sy].clone(), V[sx].clone(), W[sy].clone(), WX[sx].clone()
        ref = {"f": e.obj(x), "g": e.grad(x), "c": e.cons(x), "jac": e.jac_coord(x),
               "hess": e.hess_coord(x, y, sigma), "jv": e.jprod(x, v), "jtw": e.jtprod(x, w),
               "hv": e.hprod(x, y, sigma, v)}
        for k, t in outs.items():
            kind = ALL8[k]
            sl = slice(i, i + 1) if kind == "B" else b.slice(kind, i)
            assert torch.equal(t[sl], ref[k]), f"{tag} instance {i}: batched {k} differs from its callback"
        if lag is not None:
            assert torch.equal(lag[sx], e.lag_grad(x, y, sigma)), f"{tag} instance {i}: lag"
        if tbar is not None:
            assert torch.equal(tbar[b.slice("theta", i)], e.adjoint_theta(x, y, sigma, wx)), \
                f"{tag} instance {i}: adjoint"


FAMILIES = {
    # uneven ACOPF instances (in-place gradients, chunked J^T w and H v sums)
    "acopf": lambda: acopf_batch(6, 1000, lo=30, hi=900),
    # a variable shared by every point (dt): segments summed in parts
    "goddard": lambda: [goddard(T, s) for T, s in ((60, 1), (1500, 2), (3000, 3))],
    # root variables shared by every scenario
    "two_stage": lambda: [two_stage(S, 4, 16, s) for S, s in ((5, 1), (300, 2), (70, 3))],
    # hub variables with many objective terms: the gradient goes through a
    # reduction (long segments in parts, chunked ones, an empty hub)
    "star": lambda: [_star([700, 3], 6), _star([1500, 2, 0, 90], 7), _star([40], 8)],
}


def _star(sizes, seed):
    from test_parity_gpu import star_case
    return star_case(sizes, seed)


@pytest.mark.parametrize("family", list(FAMILIES))
@pytest.mark.parametrize("autotune,block,epl,fuse,units,graph,xcd", [
    (False, 64, 1, False, "per_callback", True, False),
    (False, 256, 3, True, "jac_hess", False, True),
    (False, 128, 8, True, "one_pass", True, True),
    (False, 256, 2, True, "separate", True, True),
    (True, 256, 4, True, "jac_hess", True, True)])
def test_every_callback_bitwise_equal_to_plain(family, autotune, block, epl, fuse, units, graph, xcd):
    _gpu()
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    wls = FAMILIES[family]()
    ems = [ExaModel(w.model) for w in wls]
    b = ExaBatch(ems, autotune=autotune, block=block, epl=epl, fuse=fuse, units=units, use_graph=graph,
                 xcd_aware=xcd)
    X, Y, V, W, WX = _inputs(b, wls)
    sigma = 0.9
    outs = {k: _nan(b, kind) for k, kind in ALL8.items()}
    for rep in range(3):  # the first call records the graph; the others replay it
        b.evaluate(X, Y, sigma, V, W, **outs)
        _check_against_plain(b, ems, X, Y, V, W, WX, sigma, outs, tag=f"{family} rep {rep}")
    # single callbacks and other selections
    for sel in (("jac",), ("hess",), ("jac", "hess"), ("f",), ("g", "c"), ("hv",), ("jtw", "jv")):
        sub = {k: _nan(b, ALL8[k]) for k in sel}
        b.evaluate(X, Y, sigma, V, W, **sub)
        _check_against_plain(b, ems, X, Y, V, W, WX, sigma, sub, tag=f"{family} {sel}")
    # the Lagrangian gradient and the parameter adjoint
    lag, tbar = _nan(b, "x"), _nan(b, "theta")
    b.evaluate(X, Y, sigma, wx=WX, lag=lag, theta_bar=tbar)
    _check_against_plain(b, ems, X, Y, V, W, WX, sigma, {}, lag=lag, tbar=tbar, tag=f"{family} lag+adj")
    lag2 = _nan(b, "x")
    b.evaluate(X, Y, sigma, lag=lag2, c=outs["c"])
    assert torch.equal(lag, lag2)
    # the store choice of the schedule changes no bit
    cbs = ("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod")
    for unstaged in (True, False):
        b.set_schedule(cbs, block, max(1, epl), fuse, units, unstaged=unstaged)
        outs = {k: _nan(b, kind) for k, kind in ALL8.items()}
        b.evaluate(X, Y, sigma, V, W, **outs)
        _check_against_plain(b, ems, X, Y, V, W, WX, sigma, outs, tag=f"{family} unstaged={unstaged}")
        assert b.schedule(cbs)["unstaged"] == int(unstaged)
    b.close()


def test_workload_slice_matches_plain_and_oracle():
    """Eight instances of the 256-instance workload (501 to 19,991 buses,
    loads perturbed): all callbacks batched, bitwise against the plain calls,
    and three of them against the oracle."""
    _gpu()
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    seeds = [1000, 1001, 1002, 1003, 1004, 1005, 1022, 1074]
    wls = [acopf_batch_instance(s) for s in seeds]
    sizes = [w.meta["nb"] for w in wls]
    assert min(sizes) >= 500 and max(sizes) <= 20000 and max(sizes) > 19000
    ems = [ExaModel(w.model) for w in wls]
    b = ExaBatch(ems, autotune=True)
    X, Y, V, W, WX = _inputs(b, wls, seed=11)
    sigma = 1.0
    outs = {k: _nan(b, kind) for k, kind in ALL8.items()}
    b.evaluate(X, Y, sigma, V, W, **outs)
    b.evaluate(X, Y, sigma, V, W, **outs)
    _check_against_plain(b, ems, X, Y, V, W, WX, sigma, outs, tag="slice")
    for i in (3, 6, 7):  # 999, 501 and 19,991 buses
        w = wls[i]
        o = OracleModel(w.model)
        sx, sy = b.slice("x", i), b.slice("y", i)
        v, wv = host(V[sx]), host(W[sy])
        a = abs_oracle(o, w.x, w.y, sigma, v, wv)
        jr, hr = o.jac_coord(w.x), o.hess_coord(w.x, w.y, sigma)
        assert_close(f"slice {i} jac", host(outs["jac"][b.slice("jac", i)]), jr, column_scale(o, jr, 1))
        assert_close(f"slice {i} hess", host(outs["hess"][b.slice("hess", i)]), hr, column_scale(o, hr, 2))
        assert_close(f"slice {i} obj", host(outs["f"])[i], o.obj(w.x), a["obj"])
        assert_close(f"slice {i} grad", host(outs["g"][sx]), o.grad(w.x), a["grad"])
        assert_close(f"slice {i} cons", host(outs["c"][sy]), o.cons(w.x), a["cons"])
        assert_close(f"slice {i} jprod", host(outs["jv"][sy]), o.jprod(w.x, v), a["jprod"])
        assert_close(f"slice {i} jtprod", host(outs["jtw"][sx]), o.jtprod(w.x, wv), a["jtprod"])
        assert_close(f"slice {i} hprod", host(outs["hv"][sx]), o.hprod(w.x, w.y, sigma, v), a["hprod"])
    b.close()


def test_batch_theta_and_autograd():
    """BatchLagrangianGradient: forward and backward equal the per-instance
    LagrangianGradient bit for bit, with theta changed through the batch;
    the adjoint against the oracle and central finite differences."""
    _gpu()
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.adjoint import batch_lagrangian_gradient, lagrangian_gradient
    from paper_2608_16265_amd.batch import ExaBatch
    wls = [acopf(30, s, gb_in_theta=True) for s in (0, 1, 2)] + [acopf(57, 3, gb_in_theta=True)]
    ems = [ExaModel(w.model) for w in wls]
    b = ExaBatch(ems, autotune=False)
    X, Y, _, _, _ = _inputs(b, wls)
    th0 = np.concatenate([w.model.theta for w in wls]) * 1.1
    theta = dev(th0).requires_grad_(True)
    sigma = 0.7
    F = batch_lagrangian_gradient(theta, b, X, Y, sigma)
    rng = np.random.default_rng(8)
    wv = dev(rng.standard_normal(b.total("x")))
    (F * wv).sum().backward()
    tb = theta.grad
    for i, (w, e) in enumerate(zip(wls, ems)):
        sx, st = b.slice("x", i), b.slice("theta", i)
        th_i = dev(th0[st]).requires_grad_(True)
        Fi = lagrangian_gradient(th_i, e, X[sx].clone(), Y[b.slice("y", i)].clone(), sigma)
        assert torch.equal(F[sx], Fi)
        (Fi * wv[sx]).sum().backward()
        assert torch.equal(tb[st], th_i.grad)
        o = OracleModel(w.model)
        ref = o.adjoint_theta(w.x, w.y, sigma, host(wv[sx]), theta=th0[st])
        assert_close(f"adjoint {i}", host(tb[st]), ref, adjoint_scale(o, w.x, w.y, sigma, host(wv[sx]), th0[st]))
    # central differences of the batched forward, h = 1e-6
    h = 1e-6
    tbh = host(tb)
    for t in rng.choice(th0.size, 8, replace=False):
        tp, tm = th0.copy(), th0.copy()
        tp[t] += h
        tm[t] -= h
        with torch.no_grad():
            fp = float(batch_lagrangian_gradient(dev(tp), b, X, Y, sigma) @ wv)
            fm = float(batch_lagrangian_gradient(dev(tm), b, X, Y, sigma) @ wv)
        fd = (fp - fm) / (2 * h)
        assert abs(tbh[t] - fd) <= 1e-6 * max(1.0, abs(fd)), (t, tbh[t], fd)
    with pytest.raises(NotImplementedError):
        batch_lagrangian_gradient(theta, b, X.clone().requires_grad_(True), Y, sigma)


def test_batch_timing_and_schedule():
    _gpu()
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    wls = acopf_batch(4, 1000, lo=30, hi=300)
    ems = [ExaModel(w.model) for w in wls]
    b = ExaBatch(ems, autotune=False)
    X, Y, V, W, WX = _inputs(b, wls)
    outs = {k: _nan(b, kind) for k, kind in ALL8.items()}
    b.set_schedule(("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod"), 128, 2, True,
                   "per_callback")
    b.timing(True)
    for _ in range(5):
        b.evaluate(X, Y, 1.0, V, W, **outs)
    t = b.timing_read()
    b.timing(False)
    assert t["calls"] == 5 and t["eval_us"] > 0 and t["reduce_calls"] == 5 and t["reduce_us"] > 0
    sch = b.schedule(("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod"))
    assert sch["block"] == 128 and sch["points_per_lane"] == 2 and sch["units"] == "per_callback"
    kb = b.kernel_bytes(("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod"))
    assert kb["eval_write"] >= 8 * (b.total("jac") + b.total("hess"))
    _check_against_plain(b, ems, X, Y, V, W, WX, 1.0, outs, tag="timed")


def test_batch_rejects_bad_calls():
    _gpu()
    from paper_2608_16265_amd import ExaError, ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    from exa_modeling.generators import rosenbrock
    with pytest.raises(ExaError):
        ExaBatch([ExaModel(acopf(30, 0).model), ExaModel(rosenbrock(10).model)])
    wls = acopf_batch(2, 1000, lo=30, hi=60)
    b = ExaBatch([ExaModel(w.model) for w in wls], autotune=False)
    X, Y, V, W, WX = _inputs(b, wls)
    with pytest.raises(ExaError):  # the Lagrangian gradient with the gradient in one call
        b.evaluate(X, Y, 1.0, g=_nan(b, "x"), lag=_nan(b, "x"))
    with pytest.raises(ValueError):
        b.evaluate(X, Y, 1.0, jac=torch.zeros(3, dtype=torch.float64, device="cuda:0"))


def test_instances_that_disagree_on_hv_references_stored_by_the_kernel():
    """A data set whose reference z[i] is its variables' only H v entry in
    some instances (i a permutation) and not in others (i with repeats):
    each instance's bit picks the kernel's own store or the reduction, in
    one launch, and every output equals the instance's own callbacks bit
    for bit."""
    _gpu()
    from exa_modeling import DataSet, Model, exp, sin
    from exa_modeling.generators import Workload
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch

    def inst(n, repeats, seed):
        rng = np.random.default_rng(seed)
        m = Model("hvd")
        x = m.add_var(n + 1)
        z = m.add_var(n)
        i = rng.integers(0, n, n) if repeats else rng.permutation(n)
        d = DataSet(n, i=i, j=np.arange(n), c=rng.uniform(0.5, 2.0, n))
        m.add_obj(d.c * z[d.i] ** 2 + x[d.j] * x[d.j + 1], d)
        m.add_con(exp(x[d.j]) * sin(z[d.i]), d)
        return Workload(m, rng.uniform(-1, 1, 2 * n + 1), rng.standard_normal(n), 1.0)
    wls = [inst(300, False, 1), inst(200, True, 2), inst(500, False, 3)]
    ems = [ExaModel(w.model) for w in wls]
    # the first instance's code stores z[i] (the batch runs it), then the
    # first instance's code does not (the batch compiles code that may)
    for order in ([0, 1, 2], [1, 0, 2]):
        sub = [ems[i] for i in order]
        b = ExaBatch(sub, autotune=False, units="per_callback")
        X, Y, V, W, WX = _inputs(b, [wls[i] for i in order])
        outs = {k: _nan(b, kind) for k, kind in ALL8.items()}
        b.evaluate(X, Y, 1.0, V, W, **outs)
        _check_against_plain(b, sub, X, Y, V, W, WX, 1.0, outs, tag=f"hvd{order}")
    # and each instance's own callbacks (H v among them) against the oracle
    from test_parity_gpu import check_all
    for i, (w, em) in enumerate(zip(wls, ems)):
        check_all(w, em, tag=f"hvd{i} ")


def test_instances_that_disagree_on_identity_columns():
    """An index column that is 0, 1, ..., n-1 in some instances and permuted
    in others: the batch runs code of its own that loads the column, and
    every output still equals each instance's own callbacks bit for bit."""
    _gpu()
    from exa_modeling import DataSet, Model, exp, sin
    from exa_modeling.generators import Workload
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch

    def inst(n, perm, seed):
        rng = np.random.default_rng(seed)
        m = Model("ident")
        x = m.add_var(n + 1)
        i = rng.permutation(n) if perm else np.arange(n)
        d = DataSet(n, i=i, c=rng.uniform(0.5, 2.0, n))
        m.add_obj(d.c * x[d.i] ** 2, d)
        m.add_con(exp(x[d.i]) * sin(x[d.i + 1]), d)
        return Workload(m, rng.uniform(-1, 1, n + 1), rng.standard_normal(n), 1.0)
    wls = [inst(300, False, 1), inst(200, True, 2), inst(500, False, 3)]
    ems = [ExaModel(w.model) for w in wls]
    b = ExaBatch(ems, autotune=False, units="per_callback")
    X, Y, V, W, WX = _inputs(b, wls)
    outs = {k: _nan(b, kind) for k, kind in ALL8.items()}
    b.evaluate(X, Y, 1.0, V, W, **outs)
    _check_against_plain(b, ems, X, Y, V, W, WX, 1.0, outs, tag="ident")
