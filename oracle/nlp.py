"""NLP callbacks of a pattern/data model, computed from their definitions.

Test infrastructure: see the package docstring.

Layout conventions (0-based; the paper is 1-based):

* constraint rows: base blocks in declaration order, row ``o0 + k`` for data
  point k of a base pattern; an augmentation adds to row
  ``o0(target) + rowcol[k] + row_off`` (eq. simd:con, Sec. 3.3.2);
* Jacobian COO: base and augmentation patterns in declaration order; data
  point k of pattern P owns entries ``o1 + k*o1step + s`` for its unique
  variable slots s (Sec. 5.3.2, write position o1 + (k-1) o1step + comp1);
* Hessian COO: all patterns in declaration order, ``o2 + k*o2step + s`` over
  the unique pairs, stored as (max, min) of the resolved global indices
  (lower triangle, Sec. 5.2.2);
* values: entry (a, b) holds w * d2T/dx_a dx_b with w = sigma for objective
  patterns and w = y[row] otherwise (Sec. 2.1.3 hess_coord); when two
  different references a != b resolve to the same variable the entry holds
  twice the mixed derivative, so that summing duplicates reproduces the true
  Hessian.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp

from . import rules, taylor

CHUNK = 1 << 15


@dataclass
class _Pat:
    kind: str
    tree: object
    ndata: int
    icols: dict
    fcols: dict
    vslots: list          # unique var keys, first-visit order
    pslots: list          # unique param keys
    hslots: list          # unique pairs (slot index a, slot index b)
    comp1: list
    comp2: list
    o0: int = 0           # first row (con) / first term (obj) / first aug term
    o1: int = 0
    o2: int = 0
    og: int = 0           # first gradient-buffer entry (obj)
    target_o0: int = -1
    row_col: str = None
    row_off: int = 0


class OracleModel:
    def __init__(self, model):
        self.model = model
        self.nvar = model.nvar
        self.ntheta = model.ntheta
        self.pats: List[_Pat] = []
        con_off = model.con_offsets()
        o1 = o2 = og = aa = tt = 0
        for p in model.patterns:
            tree = rules.simplify(rules.from_nodes(p.nodes()))
            raw1 = rules.first_order_visits(tree)
            v_uniq, comp1 = rules.compress(raw1)
            raw2 = rules.second_order_visits(tree)
            h_uniq, comp2 = rules.compress(raw2, pairs=True)
            hslots = [(v_uniq.index(a), v_uniq.index(b)) for (a, b) in h_uniq]
            p_uniq, _ = rules.compress([q.key() for q in rules.param_leaves(tree)])
            P = _Pat(p.kind, tree, p.ndata, p.data.icols, p.data.fcols,
                     v_uniq, p_uniq, hslots, comp1, comp2)
            P.o2 = o2
            o2 += p.ndata * len(hslots)
            if p.kind == "obj":
                P.o0, tt = tt, tt + p.ndata
                P.og = og
                og += p.ndata * len(v_uniq)
            else:
                P.o1 = o1
                o1 += p.ndata * len(v_uniq)
                if p.kind == "aug":
                    P.o0, aa = aa, aa + p.ndata
            self.pats.append(P)
        # base-row offsets by declaration order
        for P, p, i in zip(self.pats, model.patterns, range(len(self.pats))):
            if p.kind == "con":
                P.o0 = con_off[i]
            elif p.kind == "aug":
                P.target_o0 = con_off[p.target]
                P.row_col, P.row_off = p.row_col, p.row_off
        self.ncon = model.ncon
        self.nnzj, self.nnzh, self.nnzg = o1, o2, og

    # ------------------------------------------------------------------ dims
    def dims(self):
        return self.nvar, self.ncon, self.nnzj, self.nnzh

    def bounds(self):
        m = self.model
        return m.xl, m.xu, m.lcon, m.ucon

    # ------------------------------------------------------------- helpers
    def _index(self, P, key, ks):
        op, col, off = key
        if col is None:
            return np.full(ks.size, off, dtype=np.int64)
        return P.icols[col][ks].astype(np.int64) + off

    def _rows(self, P, ks):
        if P.kind == "con":
            return P.o0 + ks
        return P.target_o0 + P.icols[P.row_col][ks].astype(np.int64) + P.row_off

    def _leaf_fn(self, P, ks, x, theta, with_params):
        nv = len(P.vslots)

        def leaf(node):
            if node.op == "const":
                return node.value, -1
            if node.op == "data":
                return P.fcols[node.col][ks], -1
            if node.op == "var":
                return x[self._index(P, node.key(), ks)], P.vslots.index(node.key())
            if node.op == "param":
                val = theta[self._index(P, node.key(), ks)]
                return val, (nv + P.pslots.index(node.key())) if with_params else -1
            raise ValueError(node.op)
        return leaf

    def _chunks(self, P):
        for s in range(0, P.ndata, CHUNK):
            yield np.arange(s, min(P.ndata, s + CHUNK))

    def _taylor(self, P, ks, x, theta, with_params=False, dtype=np.float64):
        m = len(P.vslots) + (len(P.pslots) if with_params else 0)
        return taylor.evaluate(P.tree, self._leaf_fn(P, ks, x, theta, with_params), m, ks.size, dtype)

    def _theta(self, theta):
        return self.model.theta if theta is None else np.asarray(theta, dtype=np.float64)

    def pattern_values(self, i, x, theta=None, dtype=np.float64):
        """Values T_P(x; theta, d_k) for every data point of pattern i."""
        P = self.pats[i]
        ks = np.arange(P.ndata)
        th = self._theta(theta)
        return taylor.evaluate_value(P.tree, self._leaf_fn(P, ks, x, th, False), ks.size, dtype)

    # ------------------------------------------------------------ callbacks
    def obj(self, x, theta=None, dtype=np.float64):
        tot = sum(np.sum(self.pattern_values(i, x, theta, dtype))
                  for i, P in enumerate(self.pats) if P.kind == "obj")
        return float(tot) if dtype == np.float64 else dtype(tot)

    def cons(self, x, theta=None, dtype=np.float64):
        c = np.zeros(self.ncon, dtype=dtype)
        for i, P in enumerate(self.pats):
            if P.kind == "obj" or P.ndata == 0:
                continue
            vals = self.pattern_values(i, x, theta, dtype)
            np.add.at(c, self._rows(P, np.arange(P.ndata)), vals)
        return c

    def grad(self, x, theta=None, dtype=np.float64):
        g = np.zeros(self.nvar, dtype=dtype)
        th = self._theta(theta)
        for P in self.pats:
            if P.kind != "obj":
                continue
            for ks in self._chunks(P):
                tay = self._taylor(P, ks, x, th, dtype=dtype)
                for s, key in enumerate(P.vslots):
                    np.add.at(g, self._index(P, key, ks), tay.g[:, s])
        return g

    def jac_structure(self):
        rows = np.zeros(self.nnzj, dtype=np.int32)
        cols = np.zeros(self.nnzj, dtype=np.int32)
        for P in self.pats:
            if P.kind == "obj":
                continue
            ks = np.arange(P.ndata)
            step = len(P.vslots)
            r = self._rows(P, ks)
            for s, key in enumerate(P.vslots):
                pos = P.o1 + ks * step + s
                rows[pos] = r
                cols[pos] = self._index(P, key, ks)
        return rows, cols

    def jac_coord(self, x, theta=None, dtype=np.float64):
        """Data point k of constraint or augmentation pattern P owns entries
        o1 + k*o1step + s (Sec. 5.3.2); their values are the pattern's
        jac_block at k, so the full array and the sampled blocks come from
        one code path."""
        vals = np.zeros(self.nnzj, dtype=dtype)
        for i, P in enumerate(self.pats):
            if P.kind == "obj":
                continue
            step = len(P.vslots)
            for ks in self._chunks(P):
                blk = self.jac_block(i, ks, x, theta, dtype)
                for s in range(step):
                    vals[P.o1 + ks * step + s] = blk[:, s]
        return vals

    def hess_structure(self):
        rows = np.zeros(self.nnzh, dtype=np.int32)
        cols = np.zeros(self.nnzh, dtype=np.int32)
        for P in self.pats:
            ks = np.arange(P.ndata)
            step = len(P.hslots)
            for s, (a, b) in enumerate(P.hslots):
                ga = self._index(P, P.vslots[a], ks)
                gb = self._index(P, P.vslots[b], ks)
                pos = P.o2 + ks * step + s
                rows[pos] = np.maximum(ga, gb)
                cols[pos] = np.minimum(ga, gb)
        return rows, cols

    def _weights(self, P, ks, y, sigma, dtype=np.float64):
        if P.kind == "obj":
            return np.full(ks.size, sigma, dtype=dtype)
        return np.asarray(y, dtype=dtype)[self._rows(P, ks)]

    def hess_coord(self, x, y, sigma=1.0, theta=None, dtype=np.float64):
        """Data point k of pattern P owns entries o2 + k*o2step + s (Sec.
        5.3.2); their values are the pattern's hess_block at k."""
        vals = np.zeros(self.nnzh, dtype=dtype)
        for i, P in enumerate(self.pats):
            step = len(P.hslots)
            if step == 0:
                continue
            for ks in self._chunks(P):
                blk = self.hess_block(i, ks, x, y, sigma, theta, dtype)
                for s in range(step):
                    vals[P.o2 + ks * step + s] = blk[:, s]
        return vals

    # ------------------------------------------------------------ products
    def jac_matrix(self, x, theta=None, dtype=np.float64):
        r, c = self.jac_structure()
        return sp.coo_matrix((self.jac_coord(x, theta, dtype), (r, c)), shape=(self.ncon, self.nvar))

    def hess_matrix(self, x, y, sigma=1.0, theta=None, dtype=np.float64):
        """Full symmetric Hessian of the Lagrangian from the lower-triangle COO."""
        r, c = self.hess_structure()
        L = sp.coo_matrix((self.hess_coord(x, y, sigma, theta, dtype), (r, c)),
                          shape=(self.nvar, self.nvar)).tocsr()
        return L + L.T - sp.diags(L.diagonal())

    def jprod(self, x, v, theta=None, dtype=np.float64):
        return self.jac_matrix(x, theta, dtype) @ np.asarray(v, dtype=dtype)

    def jtprod(self, x, w, theta=None, dtype=np.float64):
        return self.jac_matrix(x, theta, dtype).T @ np.asarray(w, dtype=dtype)

    def hprod(self, x, y, sigma, v, theta=None, dtype=np.float64):
        return self.hess_matrix(x, y, sigma, theta, dtype) @ np.asarray(v, dtype=dtype)

    def grad_lagrangian(self, x, y, sigma=1.0, theta=None):
        """sigma * grad f + J^T y."""
        return sigma * self.grad(x, theta) + self.jtprod(x, y, theta)

    def adjoint_theta(self, x, y, sigma, w, theta=None):
        """(d grad_x L / d theta)^T w: for every pattern instance,
        weight * sum_a w[col_a] * d2T/dx_a dtheta_t, added into theta_t."""
        th = self._theta(theta)
        out = np.zeros(self.ntheta)
        w = np.asarray(w, dtype=np.float64)
        for P in self.pats:
            if not P.pslots or not P.vslots:
                continue
            nv = len(P.vslots)
            for ks in self._chunks(P):
                tay = self._taylor(P, ks, x, th, with_params=True)
                wt = self._weights(P, ks, y, sigma)
                for t, pkey in enumerate(P.pslots):
                    acc = np.zeros(ks.size)
                    for a, vkey in enumerate(P.vslots):
                        acc += w[self._index(P, vkey, ks)] * tay.h[:, a, nv + t]
                    np.add.at(out, self._index(P, pkey, ks), wt * acc)
        return out

    # ------------------------------------------------- values at sample points
    def jac_block(self, i, ks, x, theta=None, dtype=np.float64):
        """Jacobian values (len(ks), o1step) of pattern i at data points ks:
        column s is dT/dx of the s-th unique variable reference, summed over
        every leaf of that reference (the within-tree merge of Sec. 5.2.2).
        ``dtype`` np.longdouble gives the extended-precision reference."""
        P = self.pats[i]
        ks = np.asarray(ks, dtype=np.int64)
        return self._taylor(P, ks, x, self._theta(theta), dtype=dtype).g.copy()

    def hess_block(self, i, ks, x, y, sigma=1.0, theta=None, dtype=np.float64):
        """Hessian values (len(ks), o2step) of pattern i at data points ks:
        column s is w * d2T/dx_a dx_b for the s-th unique pair (a, b), with w
        = sigma for an objective pattern and y of the point's row otherwise
        (Sec. 2.1.3); a cross pair whose two references resolve to the same
        variable holds twice the mixed derivative, so that summing duplicate
        COO entries reproduces the Hessian."""
        P = self.pats[i]
        ks = np.asarray(ks, dtype=np.int64)
        tay = self._taylor(P, ks, x, self._theta(theta), dtype=dtype)
        w = self._weights(P, ks, y, sigma, dtype)
        out = np.zeros((ks.size, len(P.hslots)), dtype=dtype)
        for s, (a, b) in enumerate(P.hslots):
            v = w * tay.h[:, a, b]
            if a != b:
                same = (self._index(P, P.vslots[a], ks) == self._index(P, P.vslots[b], ks))
                v = np.where(same, 2 * v, v)
            out[:, s] = v
        return out

    # ------------------------------------------------------- introspection
    def probe(self, i):
        """First/second-order visit lists and compressor maps of pattern i."""
        P = self.pats[i]
        return dict(raw1=rules.first_order_visits(P.tree), comp1=P.comp1, o1step=len(P.vslots),
                    raw2=rules.second_order_visits(P.tree), comp2=P.comp2, o2step=len(P.hslots))

    def local_hessians(self, i, x, theta=None):
        """Full local Hessians (ndata, k, k) of pattern i over its var slots."""
        P = self.pats[i]
        return self._taylor(P, np.arange(P.ndata), x, self._theta(theta)).h
