"""exa_hprod_noalloc (the H v entry point that allocates nothing) through
the C ABI, against exa_hprod on the same inputs: two calls in a row, the
second with a smaller model, both bit for bit; the size limit is refused
on the host."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from exa_modeling.generators import acopf, rosenbrock
from parity_util import dev

pytestmark = pytest.mark.gpu


def _call(lib_fn, em, X, Y, sigma, V, out):
    return lib_fn(em.handle, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), C.c_double(sigma),
                  C.c_void_p(V.data_ptr()), C.c_void_p(out.data_ptr()), None)


def _case(w, seed):
    from paper_2608_16265_amd import ExaModel
    em = ExaModel(w.model)
    rng = np.random.default_rng(seed)
    y = w.y if w.y.size == em.ncon else rng.standard_normal(em.ncon)
    return em, dev(w.x), dev(y), dev(rng.standard_normal(em.nvar))


def test_hprod_noalloc_matches_hprod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_16265_amd import _lib
    from test_parity_gpu import star_case
    lib = _lib.LIB
    # a large model with long segments (part sums in the array), then a small one
    for w, seed in ((star_case([5000, 1025, 700, 3, 0, 2100], 8), 1), (acopf(600, 7), 2), (acopf(30, 0), 3)):
        em, X, Y, V = _case(w, seed)
        ref = torch.full((em.nvar,), float("nan"), dtype=torch.float64, device="cuda:0")
        got = torch.full((em.nvar,), float("nan"), dtype=torch.float64, device="cuda:0")
        assert _call(lib.exa_hprod, em, X, Y, 0.7, V, ref) == _lib.EXA_OK
        assert _call(lib.exa_hprod_noalloc, em, X, Y, 0.7, V, got) == _lib.EXA_OK, lib.exa_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        # again, with the array holding the previous call's contents
        got2 = torch.full_like(got, float("nan"))
        assert _call(lib.exa_hprod_noalloc, em, X, Y, 0.7, V, got2) == _lib.EXA_OK
        torch.cuda.synchronize()
        assert torch.equal(got2, ref)
        em.close()


def test_hprod_noalloc_refuses_models_beyond_its_array():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_16265_amd import _lib
    lib = _lib.LIB
    w = rosenbrock(2_500_000, 0)  # 2 curved slots per point: about 5e6 contributions
    em, X, Y, V = _case(w, 4)
    out = torch.zeros(em.nvar, dtype=torch.float64, device="cuda:0")
    assert _call(lib.exa_hprod_noalloc, em, X, Y, 1.0, V, out) == _lib.EXA_EINVAL
    assert b"work space" in lib.exa_last_error()
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out)) == 0  # nothing launched
    em.close()
