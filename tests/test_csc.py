"""Compressed sparse columns (the solver-side compression of Sec. 5.2).

CPU: the oracle's compression pinned against a hand-worked example, a dense
brute force and scipy's COO-to-CSC conversion (a library routine), and the
library's host analysis against the oracle's, bit for bit.  GPU: compressed
values from the device COO values against the oracle's compression of the
oracle's COO values, and their determinism.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from exa_modeling.generators import acopf, goddard, pde, rosenbrock
from oracle import OracleModel
from oracle.csc import csc_structure, csc_values
from parity_util import assert_close, column_scale, dev, host
from test_parity_gpu import aliasing_case, empty_pattern_case, star_case


def test_oracle_csc_hand_example():
    # entries (row, col): (1,0) (0,0) (1,0) (2,2) (0,0): column 0 holds rows
    # 0 and 1 (each twice), column 1 nothing, column 2 row 2
    rows, cols = [1, 0, 1, 2, 0], [0, 0, 0, 2, 0]
    vals = [1.0, 10.0, 100.0, 1000.0, 10000.0]
    colptr, rowval = csc_structure(rows, cols, 3)
    assert colptr.tolist() == [0, 2, 2, 3]
    assert rowval.tolist() == [0, 1, 2]
    assert csc_values(rows, cols, vals, 3).tolist() == [10010.0, 101.0, 1000.0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_oracle_csc_against_dense_and_scipy(seed):
    rng = np.random.default_rng(seed)
    nr, nc, nnz = 9, 7, 60
    rows, cols = rng.integers(0, nr, nnz), rng.integers(0, nc, nnz)
    vals = rng.integers(-50, 50, nnz).astype(np.float64)  # exact sums in any order
    colptr, rowval = csc_structure(rows, cols, nc)
    got = csc_values(rows, cols, vals, nc)
    dense = np.zeros((nr, nc))
    seen = np.zeros((nr, nc), dtype=bool)
    for r, c, v in zip(rows, cols, vals):
        dense[r, c] += v
        seen[r, c] = True
    for j in range(nc):
        rr = rowval[colptr[j]:colptr[j + 1]]
        assert rr.tolist() == sorted(np.flatnonzero(seen[:, j]).tolist())
        assert np.array_equal(got[colptr[j]:colptr[j + 1]], dense[rr, j])
    ref = sp.coo_matrix((vals, (rows, cols)), shape=(nr, nc)).tocsc()
    ref.sum_duplicates()
    ref.sort_indices()
    # scipy drops nothing here: every structural pair is kept even when it sums to zero
    assert np.array_equal(ref.indptr, colptr) and np.array_equal(ref.indices, rowval)
    assert np.array_equal(ref.data, got)


CASES = {
    "rosen7": lambda: rosenbrock(7, 2),
    "acopf30": lambda: acopf(30, 0),
    "pde8": lambda: pde(8, 3),
    "goddard40": lambda: goddard(40, 1),
    "alias": aliasing_case,          # pairs that alias at run time: duplicates inside a pattern
    "empty": empty_pattern_case,
    "star": lambda: star_case([700, 3, 0, 90], 6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_host_csc_structure_matches_oracle(name):
    from paper_2608_16265_amd import ExaModel
    w = CASES[name]()
    em = ExaModel(w.model, host_only=True)
    o = OracleModel(w.model)
    for which, (r, c) in (("jac", o.jac_structure()), ("hess", o.hess_structure())):
        colptr, rowval = em.csc_structure(which)
        rp, rv = csc_structure(r, c, o.nvar)
        assert np.array_equal(colptr, rp), f"{name} {which} colptr"
        assert np.array_equal(rowval, rv), f"{name} {which} rowval"


def test_csc_bad_arguments():
    from paper_2608_16265_amd import ExaModel, _lib
    import ctypes as C
    em = ExaModel(rosenbrock(5).model, host_only=True)
    nnz = C.c_int64()
    assert _lib.LIB.exa_csc_dims(em.handle, 2, C.byref(nnz)) != 0
    assert _lib.LIB.exa_csc_dims(None, 0, C.byref(nnz)) != 0
    assert _lib.LIB.exa_csc_dims(em.handle, 0, None) != 0
    assert _lib.LIB.exa_csc_values(em.handle, 1, None, None, None) != 0  # host-only: no device


GPU_CASES = dict(CASES, acopf600=lambda: acopf(600, 7), pde50=lambda: pde(50, 5),
                 goddard_long=lambda: goddard(2000, 3),
                 star_long=lambda: star_case([1500, 2], 7))  # 1,500 duplicates of one Hessian entry: parts


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(GPU_CASES))
def test_csc_values_match_oracle(name):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_16265_amd import ExaModel
    w = GPU_CASES[name]()
    em = ExaModel(w.model)
    o = OracleModel(w.model)
    X, Y = dev(w.x), dev(w.y)
    for which, (r, c), ref_coo, order, gpu_coo in (
            ("jac", o.jac_structure(), o.jac_coord(w.x), 1, lambda: em.jac_coord(X)),
            ("hess", o.hess_structure(), o.hess_coord(w.x, w.y, w.sigma), 2,
             lambda: em.hess_coord(X, Y, w.sigma))):
        coo = gpu_coo()
        got = em.csc_values(which, coo)
        ref = csc_values(r, c, ref_coo, o.nvar)
        scale = csc_values(r, c, column_scale(o, ref_coo, order), o.nvar)
        assert_close(f"{name} {which} csc", host(got), ref, scale)
        # the same sums of the device's own COO values (the device adds long
        # sums in chunks, so only to rounding of the absolute sum)
        hc = host(coo)
        assert_close(f"{name} {which} csc of device coo", host(got), csc_values(r, c, hc, o.nvar),
                     csc_values(r, c, np.abs(hc), o.nvar), rtol=1e-14)
        again = [host(em.csc_values(which, coo)) for _ in range(3)]
        for a in again:
            assert np.array_equal(a, host(got)), f"{name} {which} csc repeat"
