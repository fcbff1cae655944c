"""Batched evaluation: every instance's slice is bit-identical to the plain
per-instance call, for uneven instance sizes, all schedules."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from exa_modeling.generators import acopf, acopf_batch
from oracle import OracleModel
from parity_util import assert_close, column_scale, dev, host

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("autotune,epl,grid,graph,fuse,xcd,sep", [
    (False, 1, 64, True, False, False, True), (False, 8, 0, False, True, False, False),
    (False, 2, 16, True, False, True, False), (False, 3, 24, True, True, True, True),
    (True, 4, 0, True, True, True, False),
    # one workgroup per tile: padded XCD bins, and the plain tile order
    (False, 1, -1, True, True, True, False), (False, 2, -1, False, False, False, True)])
def test_batch_bitwise_equal_to_plain(autotune, epl, grid, graph, fuse, xcd, sep):
    _gpu()
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    wls = acopf_batch(6, 1000, lo=30, hi=900)
    ems = [ExaModel(w.model) for w in wls]
    b = ExaBatch(ems, autotune=autotune, epl=epl, grid=grid, use_graph=graph, fuse=fuse,
                 xcd_aware=xcd, separate=sep)
    X = b.concat_x([w.x for w in wls])
    Y = b.concat_y([w.y for w in wls])
    J = torch.full((b.total("jac"),), np.nan, dtype=torch.float64, device="cuda:0")
    H = torch.full((b.total("hess"),), np.nan, dtype=torch.float64, device="cuda:0")
    for rep in range(3):  # graph replays
        b.eval(X, Y, 0.9, J, H)
        torch.cuda.synchronize()
        off = b.offsets()
        for i, (w, e) in enumerate(zip(wls, ems)):
            x, y = dev(w.x), dev(w.y)
            assert torch.equal(J[off[i, 2]:off[i + 1, 2]], e.jac_coord(x))
            assert torch.equal(H[off[i, 3]:off[i + 1, 3]], e.hess_coord(x, y, 0.9))
    # jac only / hess only
    J2 = torch.zeros_like(J)
    b.eval(X, Y, 0.9, J2, None)
    assert torch.equal(J, J2)
    H2 = torch.zeros_like(H)
    b.eval(X, Y, 0.9, None, H2)
    assert torch.equal(H, H2)
    # and against the oracle for one instance
    o = OracleModel(wls[2].model)
    off = b.offsets()
    hr = o.hess_coord(wls[2].x, wls[2].y, 0.9)
    assert_close("batch hess", host(H)[off[2, 3]:off[3, 3]], hr, column_scale(o, hr, 2))
    b.close()


def test_batch_rejects_different_formulations():
    _gpu()
    from paper_2608_16265_amd import ExaModel, ExaError
    from paper_2608_16265_amd.batch import ExaBatch
    from exa_modeling.generators import rosenbrock
    with pytest.raises(ExaError):
        ExaBatch([ExaModel(acopf(30, 0).model), ExaModel(rosenbrock(10).model)])
