"""exa_eval (several callbacks at one point in one launch) against the single
callbacks, bit for bit, over every selection that matters, plus bound calls
and argument errors.  The single callbacks are themselves checked against
the oracle in test_parity_gpu.py.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from exa_modeling.generators import acopf, goddard, pde, rosenbrock, two_stage
from parity_util import dev, host
from test_parity_gpu import aliasing_case, empty_pattern_case, single_point_case, star_case

pytestmark = pytest.mark.gpu

CASES = {
    "rosen5": lambda: rosenbrock(5, 1),          # gradient through the buffer
    "rosen3000": lambda: rosenbrock(3000, 2),    # objective over two tiles
    "acopf30": lambda: acopf(30, 0),             # in-place gradient, augmentations
    "acopf600": lambda: acopf(600, 7),           # rows with more than four terms
    "pde50": lambda: pde(50, 5),
    "alias": aliasing_case,
    "empty": empty_pattern_case,
    "single": single_point_case,
    "star": lambda: star_case([700, 400, 3, 0, 90], 6),  # chunked segment sums
    "goddard": lambda: goddard(60, 1),
    "goddard_long": lambda: goddard(2000, 3),  # long segments: part sums added by a second launch
    "two_stage": lambda: two_stage(300, 4, 16, 1),
}
FIELD = {"obj": "f", "grad": "g", "cons": "c", "jac": "jac", "hess": "hess", "jprod": "jv",
         "jtprod": "jtw", "hprod": "hv"}
ALL = tuple(FIELD)
MASKS = [ALL, ("obj", "grad", "cons", "jac", "hess"), ("jprod", "jtprod", "hprod"), ("jac",), ("hess",),
         ("obj", "grad"), ("cons", "jprod"), ("grad", "jtprod", "hprod")] + [(cb,) for cb in ALL]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(w, em, seed=0):
    rng = np.random.default_rng(seed)
    return (dev(w.x), dev(w.y), float(w.sigma), dev(rng.standard_normal(em.nvar)),
            dev(rng.standard_normal(em.ncon)))


def _singles(em, X, Y, sig, V, W):
    return {"f": host(em.obj(X)), "g": host(em.grad(X)), "c": host(em.cons(X)), "jac": host(em.jac_coord(X)),
            "hess": host(em.hess_coord(X, Y, sig)), "jv": host(em.jprod(X, V)), "jtw": host(em.jtprod(X, W)),
            "hv": host(em.hprod(X, Y, sig, V))}


def _nan_like(a):
    return torch.full((a.size,), float("nan"), dtype=torch.float64, device="cuda:0")


@pytest.mark.parametrize("autotune,per_mode", [(False, False), (False, True), (True, False)])
@pytest.mark.parametrize("name", list(CASES))
def test_eval_is_bitwise_equal_to_single_callbacks(name, autotune, per_mode):
    """Per-callback tiles (the untuned default) and one-pass units (every
    selected callback of a point from one set of loads) give the single
    callbacks' bits."""
    _need_gpu()
    from paper_2608_16265_amd import ExaModel
    w = CASES[name]()
    em = ExaModel(w.model, autotune=autotune, eval_per_mode=per_mode)
    X, Y, sig, V, W = _inputs(w, em)
    ref = _singles(em, X, Y, sig, V, W)
    for mask in MASKS:
        one_pass = mask in (ALL, ("obj", "grad", "cons", "jac", "hess"))
        for units in ([None, "one_pass"] if one_pass and not autotune else [None]):
            if units:
                em.set_eval_schedule(mask, 256, 2, True, units)
            outs = {FIELD[cb]: _nan_like(ref[FIELD[cb]]) for cb in mask}
            em.evaluate(X, Y, sig, V, W, **outs)
            for k, t in outs.items():
                got = host(t)
                assert np.array_equal(got, ref[k]), f"{name} {mask} {units}: {k} differs from its single callback"
            if not autotune:
                assert em.eval_schedule(mask)["one_pass"] == (units == "one_pass" and not per_mode), mask


def test_bound_eval_follows_in_place_updates():
    _need_gpu()
    from paper_2608_16265_amd import ExaModel
    w = acopf(600, 7)
    em = ExaModel(w.model)
    X, Y, sig, V, W = _inputs(w, em, seed=1)
    ref = _singles(em, X, Y, sig, V, W)
    outs = {k: _nan_like(v) for k, v in ref.items()}
    run = em.bind(X, Y, sig, V, W, **outs)
    before = em.counters()
    for k in range(3):
        X.copy_(dev(w.x * (1.0 + 0.01 * k)))
        Y.mul_(1.1)
        run.obj_weight = 0.5 + k
        run()
        ref = _singles(em, X, Y, run.obj_weight, V, W)
        for name, t in outs.items():
            assert np.array_equal(host(t), ref[name]), f"call {k}: {name}"
    after = em.counters()
    # each round: one exa_eval plus the eight single callbacks
    for cb in ("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod"):
        assert after[cb] - before[cb] == 6


def test_objective_bits_do_not_depend_on_the_workgroup_width():
    _need_gpu()
    from paper_2608_16265_amd import ExaModel
    w = rosenbrock(3000, 2)   # two objective tiles, the second ragged
    X = dev(w.x)
    ref = host(ExaModel(w.model).obj(X))
    for block in (64, 128, 256):
        em = ExaModel(w.model, block=block, autotune=False)
        f = torch.empty(1, dtype=torch.float64, device="cuda:0")
        g = torch.empty(em.nvar, dtype=torch.float64, device="cuda:0")
        em.evaluate(X, f=f, g=g)
        assert em.eval_schedule(("obj", "grad"))["block"] == block
        assert np.array_equal(host(f), ref), block
        assert np.array_equal(host(em.obj(X)), ref), block


def test_eval_rejects_bad_arguments():
    _need_gpu()
    from paper_2608_16265_amd import ExaModel, ExaError
    from paper_2608_16265_amd import _lib
    w = acopf(30, 0)
    em = ExaModel(w.model)
    X = dev(w.x)
    H = torch.empty(em.nnzh, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        em.evaluate(X)                       # nothing selected
    with pytest.raises(ValueError):
        em.evaluate(X, hess=H)               # y missing
    with pytest.raises(ValueError):
        em.evaluate(X, dev(w.y), hess=H[:-1])  # wrong output size
    # the C entry point itself
    for mask, note in ((0, "empty mask"), (1 << 9, "unknown bit"), (_lib.EV["obj"], "f missing")):
        a = _lib.EvalArgs()
        a.mask = mask
        a.x = X.data_ptr()
        st = _lib.LIB.exa_eval(em.handle, C.byref(a), None)
        assert st == _lib.EXA_EINVAL, note
    with pytest.raises(ExaError):
        em.eval_schedule(("cons",))          # never evaluated with this set


def test_fixed_schedule_gives_the_same_bits():
    """exa_eval_set_schedule pins a schedule (no tuning); every schedule and
    every kind of units evaluates each point with the same code, so the
    outputs do not change."""
    from paper_2608_16265_amd import ExaModel
    w = acopf(200, 3)
    rng = np.random.default_rng(4)
    ref_m = ExaModel(w.model)
    X, Y = dev(w.x), dev(w.y)
    V, W = dev(rng.standard_normal(ref_m.nvar)), dev(rng.standard_normal(ref_m.ncon))
    names = ("f", "g", "c", "jac", "hess", "jv", "jtw", "hv")
    sizes = (1, ref_m.nvar, ref_m.ncon, ref_m.nnzj, ref_m.nnzh, ref_m.ncon, ref_m.nvar, ref_m.nvar)
    field = dict(zip(("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod"), names))
    e = lambda n: torch.empty(n, dtype=torch.float64, device="cuda:0")  # noqa: E731
    ref = {k: e(n) for k, n in zip(names, sizes)}
    ref_m.evaluate(X, Y, 0.9, V, W, **ref)
    every = ("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod")
    ipm = ("obj", "grad", "cons", "jac", "hess")
    for cbs, block, epl, fused, units, expect in (
            (every, 64, 3, False, "per_callback", (0, 0)), (every, 256, 1, True, "one_pass", (1, 0)),
            (every, 128, 16, False, "jac_hess", (0, 1)), (ipm, 128, 2, True, "per_callback", (0, 0)),
            (ipm, 64, 1, False, "one_pass", (1, 0)), (("jac", "hess"), 256, 4, False, "per_callback", (0, 0)),
            (("jac", "hess"), 64, 2, True, "one_pass", (0, 1)),   # no one-pass units: JH units
            (("jac", "jprod"), 128, 1, False, "jac_hess", (0, 0))):  # no Hessian: per callback
        em = ExaModel(w.model, autotune=True)
        em.set_eval_schedule(cbs, block, epl, fused, units)
        out = {field[cb]: e(n) for cb, n in zip(every, sizes) if cb in cbs}
        em.evaluate(X, Y, 0.9, V, W, **out)
        sch = em.eval_schedule(cbs)
        assert (sch["block"], sch["points_per_lane"]) == (block, epl)
        assert (sch["one_pass"], sch["jac_hess"]) == expect, (cbs, units)
        for k, t in out.items():
            assert np.array_equal(host(t), host(ref[k])), (cbs, block, epl, fused, units, k)
    with pytest.raises(Exception):
        ref_m.set_eval_schedule(every, 96, 1)
    with pytest.raises(Exception):
        ref_m.set_eval_schedule(every, 128, 0)
    with pytest.raises(Exception):
        ref_m.set_eval_schedule(every, 128, 1, units=3)


@pytest.mark.parametrize("units", ["per_callback", "jac_hess", "one_pass"])
@pytest.mark.parametrize("name", ["acopf600", "pde50", "star", "goddard_long", "two_stage", "alias", "empty"])
def test_store_choice_and_unfused_schedules_change_no_bit(name, units):
    """Staged or each lane's own stores, fused or separate patterns (J^T w
    and H v units always hold a data set's patterns, which add their
    contributions in the lane): exa_eval gives the bits of the single
    callbacks."""
    _need_gpu()
    from paper_2608_16265_amd import ExaModel
    w = CASES[name]()
    em = ExaModel(w.model)
    X, Y, sig, V, W = _inputs(w, em, seed=3)
    ref = _singles(em, X, Y, sig, V, W)
    for mask in (ALL, ("jac", "jtprod"), ("jac", "hess", "jtprod", "hprod"), ("grad", "jac", "jtprod")):
        for fused, unstaged in ((True, False), (False, False), (True, True), (False, True)):
            em.set_eval_schedule(mask, 128, 2, fused, units, unstaged=unstaged)
            outs = {FIELD[cb]: _nan_like(ref[FIELD[cb]]) for cb in mask}
            em.evaluate(X, Y, sig, V, W, **outs)
            for k, t in outs.items():
                assert np.array_equal(host(t), ref[k]), f"{name} {mask} fused={fused} unstaged={unstaged}: {k}"
            assert em.eval_schedule(mask)["unstaged"] == int(unstaged), mask
