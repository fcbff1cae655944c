"""Helpers for comparing the GPU library with the CPU oracle.

Tolerance (values), the rule "|gpu - ref| <= 1e-12 max(|ref|, s_P)": an entry passes when
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
    """Scales for the dense outputs: every contribution counts with the
    largest magnitude in its (pattern, slot) column, so that cancellation
    inside a pattern value (g cos + b sin, p - P(v, theta) ...) is measured
    against the size of the pattern's terms, as for the COO values."""
    import scipy.sparse as sp
    out = {}
    th = o._theta(theta)
    # cons / obj: per pattern, the largest |value| over its data points
    c = np.zeros(o.ncon)
    tot_obj = 0.0
    for i, P in enumerate(o.pats):
        if P.ndata == 0:
            continue
        sP = float(np.max(np.abs(o.pattern_values(i, x, theta))))
        if P.kind == "obj":
            tot_obj += P.ndata * sP
        else:
            np.add.at(c, o._rows(P, np.arange(P.ndata)), sP)
    out["cons"] = c
    out["obj"] = tot_obj
    rj, cj = o.jac_structure()
    jv = column_scale(o, o.jac_coord(x, theta), 1)
    Ja = sp.coo_matrix((jv, (rj, cj)), shape=(o.ncon, o.nvar))
    out["jprod"] = Ja @ np.abs(v)
    out["jtprod"] = Ja.T @ np.abs(w)
    out["jtprod_y"] = Ja.T @ np.abs(y)
    rh, ch = o.hess_structure()
    hv = column_scale(o, o.hess_coord(x, y, sigma, theta), 2)
    L = sp.coo_matrix((hv, (rh, ch)), shape=(o.nvar, o.nvar)).tocsr()
    Ha = L + L.T - sp.diags(L.diagonal())
    out["hprod"] = Ha @ np.abs(v)
    # grad: per-variable sum of column maxima of the objective slots
    g = np.zeros(o.nvar)
    for P in o.pats:
        if P.kind != "obj" or P.ndata == 0:
            continue
        ks = np.arange(P.ndata)
        tay = o._taylor(P, ks, x, th)
        for s_, key in enumerate(P.vslots):
            np.add.at(g, o._index(P, key, ks), np.max(np.abs(tay.g[:, s_])))
    out["grad"] = g
    return out


def adjoint_scale(o, x, y, sigma, w, theta=None):
    """Per-entry scale for the parameter adjoint theta_bar = sum over
    pattern instances of weight * sum_a w[col_a] d2T/dx_a dtheta_t: every
    term counts with |weight| |w[col_a]| times the largest |d2T/dx_a
    dtheta_t| in its (pattern, slot pair) column, as column_scale measures
    COO values against their column."""
    th = o._theta(theta)
    out = np.zeros(o.ntheta)
    w = np.asarray(w, dtype=np.float64)
    for P in o.pats:
        if not P.pslots or not P.vslots or P.ndata == 0:
            continue
        nv = len(P.vslots)
        ks = np.arange(P.ndata)
        tay = o._taylor(P, ks, x, th, with_params=True)
        wt = np.abs(o._weights(P, ks, y, sigma))
        for t, pkey in enumerate(P.pslots):
            acc = np.zeros(ks.size)
            for a, vkey in enumerate(P.vslots):
                acc += np.abs(w[o._index(P, vkey, ks)]) * np.max(np.abs(tay.h[:, a, nv + t]))
            np.add.at(out, o._index(P, pkey, ks), wt * acc)
    return out
