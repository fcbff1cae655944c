"""Checks that pin the CPU oracle to mathematics rather than to itself.

Used by test_oracle_pins.py and by test_oracle_mutations.py (which plants
mistakes in the oracle and expects these checks to catch them).  Each check
returns the worst scaled error it saw; callers compare with a bound.
"""
import math

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


def aug_offset_closed_form(wl):
    """Callbacks of the model of ``aug_offset_case`` written out by hand.

    Row layout (eq. simd:con, Sec. 3.3.2): block A holds rows 0..2 (x_i x_{i+1}),
    block B rows 3..10 (x_r^2).  Augmentation 1 adds c_k sin(x_j) x_m to row
    3 + bus_k + 2 and augmentation 2 adds exp(x_j) to row 3 + bus_k - 1.
    Returns cons, (jac rows, cols, vals) and (hess rows, cols, vals) in the
    partially compressed order of Sec. 5.3.2, from the textbook derivatives
    only (no oracle code)."""
    d1, d2 = wl.meta["aug1"], wl.meta["aug2"]
    x, y = wl.x, wl.y
    cons = np.zeros(11)
    jr, jc, jv, hr, hc, hv = [], [], [], [], [], []
    for i in range(3):                      # block A: x_i x_{i+1}
        cons[i] = x[i] * x[i + 1]
        jr += [i, i]
        jc += [i, i + 1]
        jv += [x[i + 1], x[i]]
    for i in range(3):                      # its Hessian: the cross pair only
        hr.append(i + 1)
        hc.append(i)
        hv.append(y[i])
    for r in range(8):                      # block B: x_r^2
        cons[3 + r] = x[r] ** 2
        jr.append(3 + r)
        jc.append(r)
        jv.append(2 * x[r])
        hr.append(r)
        hc.append(r)
        hv.append(2 * y[3 + r])
    for bus, j, m, c in zip(d1["bus"], d1["j"], d1["m"], d1["c"]):
        row = 3 + int(bus) + 2
        cons[row] += c * math.sin(x[j]) * x[m]
        jr += [row, row]
        jc += [int(j), int(m)]
        jv += [c * math.cos(x[j]) * x[m], c * math.sin(x[j])]
        hr += [int(j), max(int(j), int(m))]
        hc += [int(j), min(int(j), int(m))]
        hv += [y[row] * (-c * math.sin(x[j]) * x[m]), y[row] * c * math.cos(x[j])]
    for bus, j in zip(d2["bus"], d2["j"]):
        row = 3 + int(bus) - 1
        cons[row] += math.exp(x[j])
        jr.append(row)
        jc.append(int(j))
        jv.append(math.exp(x[j]))
        hr.append(int(j))
        hc.append(int(j))
        hv.append(y[row] * math.exp(x[j]))
    return cons, (np.array(jr), np.array(jc), np.array(jv)), (np.array(hr), np.array(hc), np.array(hv))


def check_aug_offset(wl):
    """Worst relative error of the oracle against aug_offset_closed_form
    (inf when a structure array differs)."""
    o = OracleModel(wl.model)
    cons, (jr, jc, jv), (hr, hc, hv) = aug_offset_closed_form(wl)
    r, c = o.jac_structure()
    if not (np.array_equal(r, jr) and np.array_equal(c, jc)):
        return math.inf
    r, c = o.hess_structure()
    if not (np.array_equal(r, hr) and np.array_equal(c, hc)):
        return math.inf
    return max(scaled_err(o.cons(wl.x), cons), scaled_err(o.jac_coord(wl.x), jv),
               scaled_err(o.hess_coord(wl.x, wl.y, wl.sigma), hv))
