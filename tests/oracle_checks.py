"""Checks that pin the CPU oracle to mathematics rather than to itself.

Used by test_oracle_pins.py and by test_oracle_mutations.py (which plants
mistakes in the oracle and expects these checks to catch them).  Each check
returns the worst scaled error it saw; callers compare with a bound.
"""
import numpy as np

from oracle import OracleModel


def dense_jac(o, x):
    return o.jac_matrix(x).toarray()


def complex_step_jac(o, x, h=1e-30):
    """J[:, j] = Im c(x + i h e_j) / h  (complex step, exact to roundoff)."""
    J = np.zeros((o.ncon, o.nvar))
    for j in range(o.nvar):
        xc = x.astype(np.complex128)
        xc[j] += 1j * h
        J[:, j] = np.imag(o.cons(xc, dtype=np.complex128)) / h
    return J


def complex_step_grad(o, x, h=1e-30):
    g = np.zeros(o.nvar)
    for j in range(o.nvar):
        xc = x.astype(np.complex128)
        xc[j] += 1j * h
        tot = 0.0
        for i, P in enumerate(o.pats):
            if P.kind == "obj":
                tot += np.sum(np.imag(o.pattern_values(i, xc, dtype=np.complex128)))
        g[j] = tot / h
    return g


def scaled_err(a, b):
    """max |a - b| / max(1, max|b|) -- a relative error with a unit floor."""
    a, b = np.asarray(a), np.asarray(b)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def check_first_order(wl):
    o = OracleModel(wl.model)
    e1 = scaled_err(dense_jac(o, wl.x), complex_step_jac(o, wl.x)) if o.ncon else 0.0
    e2 = scaled_err(o.grad(wl.x), complex_step_grad(o, wl.x))
    return max(e1, e2)


def fd_hessian(o, x, y, sigma, h=1e-6):
    """Central differences of the oracle's Lagrangian gradient."""
    H = np.zeros((o.nvar, o.nvar))
    for j in range(o.nvar):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        H[:, j] = (o.grad_lagrangian(xp, y, sigma) - o.grad_lagrangian(xm, y, sigma)) / (2 * h)
    return H


def check_second_order(wl):
    o = OracleModel(wl.model)
    H = o.hess_matrix(wl.x, wl.y, wl.sigma).toarray()
    Hfd = fd_hessian(o, wl.x, wl.y, wl.sigma)
    return scaled_err(H, Hfd)


def check_coverage(wl, seeds=(0, 1)):
    """Every nonzero of every local Hessian sits on a structural slot, and
    every local Hessian is symmetric.  Returns the largest uncovered or
    asymmetric magnitude relative to the largest entry."""
    o = OracleModel(wl.model)
    worst = 0.0
    for seed in seeds:
        rng = np.random.default_rng(seed)
        x = wl.x + 0.01 * rng.standard_normal(wl.x.size)
        for i, P in enumerate(o.pats):
            if P.ndata == 0 or not P.vslots:
                continue
            Hl = o.local_hessians(i, x)
            scale = max(1.0, float(np.max(np.abs(Hl))))
            mask = np.zeros(Hl.shape[1:], dtype=bool)
            for a, b in P.hslots:
                mask[a, b] = mask[b, a] = True
            worst = max(worst, float(np.max(np.abs(Hl[:, ~mask]), initial=0.0)) / scale)
            worst = max(worst, float(np.max(np.abs(Hl - Hl.transpose(0, 2, 1)))) / scale)
    return worst
