"""Full compression of a partially compressed COO matrix into CSC --
TEST INFRASTRUCTURE (see the package header).

The evaluator writes the Jacobian and the Hessian's lower triangle in the
partially compressed COO layout of Sec. 5.2: entries from different patterns
or different data points that land on the same (row, col) position stay
separate.  A solver that wants compressed sparse columns sums them, and only
the sums depend on the point; the structure is analysed once (Sec. 5.2.2,
Sec. 7.2.3).

Definition written out here: one CSC entry per distinct (row, col) pair of
the COO structure, columns ascending, rows ascending within a column, value
= the sum of the COO values at every position carrying that pair, added in
ascending COO position.
"""
from __future__ import annotations

import numpy as np


def _order(rows, cols):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    # stable: equal (col, row) keys keep ascending COO position
    order = np.lexsort((rows, cols))
    r, c = rows[order], cols[order]
    first = np.ones(r.size, dtype=bool)
    first[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    return order, r, c, first


def csc_structure(rows, cols, ncol: int):
    """(colptr [ncol+1], rowval [nnz]) of the distinct pairs."""
    _, r, c, first = _order(rows, cols)
    rowval = r[first]
    colptr = np.zeros(ncol + 1, dtype=np.int64)
    np.add.at(colptr, c[first] + 1, 1)
    return np.cumsum(colptr), rowval


def csc_values(rows, cols, vals, ncol: int):
    """Values of the distinct pairs, in csc_structure's order."""
    order, r, c, first = _order(rows, cols)
    v = np.asarray(vals, dtype=np.float64)[order]
    out = np.zeros(int(first.sum()))
    slot = np.cumsum(first) - 1
    for j in range(v.size):  # ascending COO position within each slot
        out[slot[j]] += v[j]
    return out
