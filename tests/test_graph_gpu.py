"""The per-iterate calls inside a captured HIP graph (torch.cuda.CUDAGraph):
after warm-up (the first call of each selection tunes and synchronizes),
exa_eval, exa_lag_grad and exa_csc_values launch only kernels on the current
stream, so a solver can capture one iterate's evaluation and replay it.
Every replay, with the inputs changed in place between replays by eager
work, must equal the eager calls bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from exa_modeling.generators import acopf, goddard
from parity_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("make", [lambda: acopf(200, 3), lambda: goddard(2000, 3)], ids=["acopf200", "goddard2000"])
def test_captured_iterate_replays_equal_eager(make):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_16265_amd import ExaModel
    w = make()
    em = ExaModel(w.model, autotune=True)
    rng = np.random.default_rng(11)
    X, Y = dev(w.x), dev(w.y)
    V, W = dev(rng.standard_normal(em.nvar)), dev(rng.standard_normal(em.ncon))
    e = lambda n: torch.empty(n, dtype=torch.float64, device="cuda:0")  # noqa: E731
    names = ["f", "g", "c", "jac", "hess", "jv", "jtw", "hv"]
    sizes = [1, em.nvar, em.ncon, em.nnzj, em.nnzh, em.ncon, em.nvar, em.nvar]
    outs = {k: e(n) for k, n in zip(names, sizes)}
    lg = e(em.nvar)
    cj = e(int(em.csc_structure("jac")[0][-1]))
    step = em.bind(X, Y, 0.7, V, W, **outs)

    def iterate():
        step()
        em.lag_grad(X, Y, 0.7, lg)
        em.csc_values("jac", outs["jac"], cj)

    iterate()  # tunes, uploads the CSC map
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        iterate()
    x0 = w.x.copy()
    for rep in range(4):
        X.copy_(torch.as_tensor(x0 * (1.0 + 0.01 * rep), device="cuda:0"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = {k: host(t) for k, t in outs.items()}
        got["lg"], got["cj"] = host(lg), host(cj)
        iterate()  # eager, same inputs
        torch.cuda.synchronize()
        ref = {k: host(t) for k, t in outs.items()}
        ref["lg"], ref["cj"] = host(lg), host(cj)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), f"replay {rep}: {k}"
