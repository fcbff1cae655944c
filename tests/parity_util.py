"""Helpers for comparing the GPU library with the CPU oracle.

Tolerance (values): an entry passes when
    |gpu - ref| <= RTOL * max(|ref|, scale)
where ``scale`` is the magnitude the entry's rounding is measured against:
for COO values the largest |ref| in the same (pattern, slot) column, for
dense sums the sum of the absolute contributions.  RTOL = 1e-12 (FP64).
Structure and integer outputs must be identical.
"""
import numpy as np
import torch

RTOL = 1e-12


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_close(name, got, ref, scale=0.0, rtol=RTOL):
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, f"{name}: shape {got.shape} vs {ref.shape}"
    if got.size == 0:
        return
    tol = rtol * np.maximum(np.abs(ref), scale)
    err = np.abs(got - ref)
    bad = ~(err <= tol)
    same_nonfinite = ~np.isfinite(ref) & (got == ref)
    bad &= ~same_nonfinite
    if bad.any():
        i = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"{name}: {bad.sum()} of {got.size} entries off; first at {i}: "
                             f"gpu={got[i]!r} ref={ref[i]!r} tol={tol.flat[i]:.3e}")


def column_scale(o, vals, order):
    """Per-entry scale for COO values: max |ref| over the entry's (pattern,
    slot) column.  order = 1 for the Jacobian, 2 for the Hessian."""
    sc = np.zeros_like(vals)
    for P in o.pats:
        if order == 1:
            if P.kind == "obj":
                continue
            st, base = len(P.vslots), P.o1
        else:
            st, base = len(P.hslots), P.o2
        if st == 0 or P.ndata == 0:
            continue
        blk = np.abs(vals[base:base + P.ndata * st]).reshape(P.ndata, st)
        sc[base:base + P.ndata * st] = np.broadcast_to(blk.max(axis=0), blk.shape).reshape(-1)
    return sc


def abs_oracle(o, x, y, sigma, v, w, theta=None):
    """Sums of absolute contributions for the dense outputs."""
    import scipy.sparse as sp
    out = {}
    # cons: sum |terms| per row
    c = np.zeros(o.ncon)
    for i, P in enumerate(o.pats):
        if P.kind == "obj" or P.ndata == 0:
            continue
        np.add.at(c, o._rows(P, np.arange(P.ndata)), np.abs(o.pattern_values(i, x, theta)))
    out["cons"] = c
    J = o.jac_matrix(x, theta)
    Ja = sp.coo_matrix((np.abs(J.data), (J.row, J.col)), shape=J.shape)
    out["jprod"] = Ja @ np.abs(v)
    out["jtprod"] = Ja.T @ np.abs(w)
    H = o.hess_matrix(x, y, sigma, theta).tocoo()
    Ha = sp.coo_matrix((np.abs(H.data), (H.row, H.col)), shape=H.shape)
    out["hprod"] = Ha @ np.abs(v)
    # grad: sum |contributions| per variable
    g = np.zeros(o.nvar)
    th = o._theta(theta)
    for P in o.pats:
        if P.kind != "obj" or P.ndata == 0:
            continue
        ks = np.arange(P.ndata)
        tay = o._taylor(P, ks, x, th)
        for s, key in enumerate(P.vslots):
            np.add.at(g, o._index(P, key, ks), np.abs(tay.g[:, s]))
    out["grad"] = g
    out["obj"] = float(sum(np.sum(np.abs(o.pattern_values(i, x, theta)))
                           for i, P in enumerate(o.pats) if P.kind == "obj"))
    return out
