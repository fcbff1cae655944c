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

from exa_modeling.generators import acopf, pde
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
