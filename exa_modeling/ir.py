"""Pattern/data model description (paper Sec. 2.2 eq. simd, Sec. 3, Sec. 4).

A :class:`Model` holds variable blocks, parameter blocks (the shared vector
theta of eq. nlp), and an ordered list of :class:`Pattern` objects.  Each
pattern is one algebraic expression tree (Sec. 4) paired with a data set of
``ndata`` points stored column-wise (struct of arrays):

* ``kind == "obj"``: a group of objective terms (eq. simd:obj);
* ``kind == "con"``: a base constraint block, one row per data point
  (eq. simd:con, the g^(m) terms);
* ``kind == "aug"``: an augmentation of an existing constraint block; each
  data point adds its value to the row of the target block selected by an
  integer data column (the h^(n) terms, Sec. 3.3 ConstraintAugmentation).

Expression nodes (Sec. 4.2):

* leaves: ``const`` (a literal), ``data`` (a float data column of the current
  point), ``var`` (an entry of x), ``param`` (an entry of theta);
* ``var``/``param`` carry an index of the form ``icol[k] + off`` where
  ``icol`` is an integer data column, or the literal ``off`` when no column is
  given.  This is the data-dependent index of Sec. 4.2.2 restricted to one
  column plus a constant; the block offset of Sec. 3.3.1 is folded into
  ``off``;
* unary and binary operators from :data:`UNARY_OPS` / :data:`BINARY_OPS`.

Expressions are recorded as written: ``x**2`` is ``pow(x, 2)``, ``2*x`` is
``mul(2, x)``.  Rewriting is the consumer's job.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple, Union

import numpy as np

LEAF_OPS = ("const", "data", "var", "param")
UNARY_OPS = ("neg", "abs2", "inv", "sqrt", "exp", "log", "sin", "cos", "tan",
             "atan", "sinh", "cosh", "tanh", "log1p", "expm1")
BINARY_OPS = ("add", "sub", "mul", "div", "pow")


class Expr:
    """One node of a parameterized expression tree (Sec. 4.2)."""

    __slots__ = ("op", "args", "value", "col", "off")

    def __init__(self, op: str, args: Tuple["Expr", ...] = (), value: float = 0.0,
                 col: Optional[str] = None, off: int = 0):
        if op not in LEAF_OPS and op not in UNARY_OPS and op not in BINARY_OPS:
            raise ValueError(f"unknown operator {op!r}")
        self.op = op
        self.args = tuple(args)
        self.value = float(value)
        self.col = col
        self.off = int(off)

    # -- construction by operator overloading (Sec. 4.1.1) -----------------
    @staticmethod
    def lift(v: Union["Expr", float, int, "DataRef"]) -> "Expr":
        if isinstance(v, Expr):
            return v
        if isinstance(v, DataRef):
            return Expr("data", col=v.name)
        if isinstance(v, (int, float, np.integer, np.floating)) and not isinstance(v, bool):
            return Expr("const", value=float(v))
        raise TypeError(f"cannot use {type(v).__name__} in an expression")

    def _bin(self, op, other, swap=False):
        a, b = Expr.lift(self), Expr.lift(other)
        return Expr(op, (b, a) if swap else (a, b))

    def __add__(self, o): return self._bin("add", o)
    def __radd__(self, o): return self._bin("add", o, True)
    def __sub__(self, o): return self._bin("sub", o)
    def __rsub__(self, o): return self._bin("sub", o, True)
    def __mul__(self, o): return self._bin("mul", o)
    def __rmul__(self, o): return self._bin("mul", o, True)
    def __truediv__(self, o): return self._bin("div", o)
    def __rtruediv__(self, o): return self._bin("div", o, True)
    def __pow__(self, o): return self._bin("pow", o)
    def __rpow__(self, o): return self._bin("pow", o, True)
    def __neg__(self): return Expr("neg", (self,))
    def __pos__(self): return self

    def __repr__(self):
        if self.op == "const":
            return repr(self.value)
        if self.op == "data":
            return f"d.{self.col}"
        if self.op in ("var", "param"):
            s = "x" if self.op == "var" else "θ"
            if self.col is None:
                return f"{s}[{self.off}]"
            return f"{s}[d.{self.col}{self.off:+d}]"
        if len(self.args) == 1:
            return f"{self.op}({self.args[0]!r})"
        return f"{self.op}({self.args[0]!r}, {self.args[1]!r})"


def _unary(op):
    def f(u):
        return Expr(op, (Expr.lift(u),))
    f.__name__ = op
    return f


exp = _unary("exp"); log = _unary("log"); sin = _unary("sin"); cos = _unary("cos")
tan = _unary("tan"); atan = _unary("atan"); sinh = _unary("sinh"); cosh = _unary("cosh")
tanh = _unary("tanh"); sqrt = _unary("sqrt"); inv = _unary("inv"); abs2 = _unary("abs2")
log1p = _unary("log1p"); expm1 = _unary("expm1")


class DataRef:
    """A column of the current data point, ``d.name`` (Sec. 4.1.3).

    Used as a value it becomes a ``data`` leaf; used (plus an integer) as an
    index into a variable or parameter block it becomes part of that index.
    """

    __slots__ = ("name", "shift")

    def __init__(self, name: str, shift: int = 0):
        self.name = name
        self.shift = int(shift)

    def __add__(self, o):
        if isinstance(o, (int, np.integer)):
            return DataRef(self.name, self.shift + int(o))
        return Expr.lift(self) + o

    def __radd__(self, o):
        if isinstance(o, (int, np.integer)):
            return DataRef(self.name, self.shift + int(o))
        return o + Expr.lift(self)

    def __sub__(self, o):
        if isinstance(o, (int, np.integer)):
            return DataRef(self.name, self.shift - int(o))
        return Expr.lift(self) - o

    def __rsub__(self, o): return o - Expr.lift(self)
    def __mul__(self, o): return Expr.lift(self) * o
    def __rmul__(self, o): return o * Expr.lift(self)
    def __truediv__(self, o): return Expr.lift(self) / o
    def __rtruediv__(self, o): return o / Expr.lift(self)
    def __pow__(self, o): return Expr.lift(self) ** o
    def __neg__(self): return -Expr.lift(self)


class DataSet:
    """Column-wise (struct of arrays) data of one pattern (Sec. 4.1.3)."""

    def __init__(self, ndata: int, **cols):
        self.ndata = int(ndata)
        self.icols: Dict[str, np.ndarray] = {}
        self.fcols: Dict[str, np.ndarray] = {}
        for k, v in cols.items():
            a = np.asarray(v)
            if a.shape != (self.ndata,):
                raise ValueError(f"column {k!r} has shape {a.shape}, expected ({self.ndata},)")
            if np.issubdtype(a.dtype, np.integer):
                if a.size and (a.min() < -2**31 or a.max() >= 2**31):
                    raise ValueError(f"column {k!r} does not fit int32")
                self.icols[k] = np.ascontiguousarray(a, dtype=np.int32)
            else:
                self.fcols[k] = np.ascontiguousarray(a, dtype=np.float64)

    def __getattr__(self, name):
        if name.startswith("_") or name in ("ndata", "icols", "fcols"):
            raise AttributeError(name)
        if name in self.icols or name in self.fcols:
            return DataRef(name)
        raise AttributeError(f"data set has no column {name!r}")


@dataclass
class VarBlock:
    """Handle of a variable block (Sec. 3.3.1 Variable): offset and length."""
    offset: int
    length: int
    name: str = ""

    def __getitem__(self, idx) -> Expr:
        return _index_expr("var", self.offset, self.length, idx)


@dataclass
class ParBlock:
    """Handle of a parameter block (Sec. 3.3.1 Parameter)."""
    offset: int
    length: int
    name: str = ""

    def __getitem__(self, idx) -> Expr:
        return _index_expr("param", self.offset, self.length, idx)


def _index_expr(op, offset, length, idx):
    if isinstance(idx, (int, np.integer)):
        i = int(idx)
        if not 0 <= i < length:
            raise IndexError(f"index {i} outside block of length {length}")
        return Expr(op, off=offset + i)
    if isinstance(idx, DataRef):
        return Expr(op, col=idx.name, off=offset + idx.shift)
    raise TypeError("a block is indexed by an int or by a data column (+ int)")


@dataclass
class Node:
    """One entry of the post-order node list handed to the consumers.

    ``a``/``b`` are positions of the children in the list (-1 when absent).
    """
    op: str
    a: int = -1
    b: int = -1
    value: float = 0.0
    col: Optional[str] = None
    off: int = 0


@dataclass
class Pattern:
    kind: str                      # "obj" | "con" | "aug"
    expr: Expr
    data: DataSet
    name: str = ""
    lcon: Optional[np.ndarray] = None   # con: per-row bounds
    ucon: Optional[np.ndarray] = None
    target: int = -1               # aug: index (in Model.patterns) of the con block
    row_col: Optional[str] = None  # aug: row within the block = icol[k] + row_off
    row_off: int = 0

    @property
    def ndata(self) -> int:
        return self.data.ndata

    def nodes(self) -> List[Node]:
        """Post-order (children first, root last) node list of the tree.

        A Python object used at two places of an expression becomes two
        separate subtrees, so the result is always a tree, as in Sec. 4.
        """
        out: List[Node] = []

        def visit(e: Expr) -> int:
            if e.op in LEAF_OPS:
                out.append(Node(e.op, value=e.value, col=e.col, off=e.off))
                return len(out) - 1
            if len(e.args) == 1:
                a = visit(e.args[0])
                out.append(Node(e.op, a=a))
                return len(out) - 1
            a = visit(e.args[0])
            b = visit(e.args[1])
            out.append(Node(e.op, a=a, b=b))
            return len(out) - 1

        visit(self.expr)
        return out


class Model:
    """An NLP in the pattern-over-data form (Sec. 2.2, eq. simd)."""

    def __init__(self, name: str = "model"):
        self.name = name
        self.nvar = 0
        self.ntheta = 0
        self._xl: List[np.ndarray] = []
        self._xu: List[np.ndarray] = []
        self._x0: List[np.ndarray] = []
        self._theta: List[np.ndarray] = []
        self.patterns: List[Pattern] = []
        self.var_blocks: List[VarBlock] = []
        self.par_blocks: List[ParBlock] = []

    # -- declarations (Sec. 2.2.3) ------------------------------------------
    def add_var(self, n: int, lvar=-math.inf, uvar=math.inf, start=0.0, name="") -> VarBlock:
        n = int(n)
        blk = VarBlock(self.nvar, n, name)
        self._xl.append(np.broadcast_to(np.asarray(lvar, dtype=np.float64), (n,)).copy())
        self._xu.append(np.broadcast_to(np.asarray(uvar, dtype=np.float64), (n,)).copy())
        self._x0.append(np.broadcast_to(np.asarray(start, dtype=np.float64), (n,)).copy())
        self.nvar += n
        self.var_blocks.append(blk)
        return blk

    def add_par(self, values, name="") -> ParBlock:
        v = np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(-1))
        blk = ParBlock(self.ntheta, v.size, name)
        self._theta.append(v)
        self.ntheta += v.size
        self.par_blocks.append(blk)
        return blk

    def add_obj(self, expr, data: DataSet, name="") -> int:
        self.patterns.append(Pattern("obj", Expr.lift(expr), data, name))
        return len(self.patterns) - 1

    def add_con(self, expr, data: DataSet, lcon=0.0, ucon=0.0, name="") -> int:
        n = data.ndata
        lc = np.broadcast_to(np.asarray(lcon, dtype=np.float64), (n,)).copy()
        uc = np.broadcast_to(np.asarray(ucon, dtype=np.float64), (n,)).copy()
        self.patterns.append(Pattern("con", Expr.lift(expr), data, name, lcon=lc, ucon=uc))
        return len(self.patterns) - 1

    def add_con_aug(self, con: int, row: DataRef, expr, data: DataSet, name="") -> int:
        """``con[row] += expr for d in data`` (the add_con! macro of Sec. 2.2.3)."""
        if not (0 <= con < len(self.patterns)) or self.patterns[con].kind != "con":
            raise ValueError("augmentation target must be a constraint block")
        if not isinstance(row, DataRef) or row.name not in data.icols:
            raise ValueError("augmentation row must be an integer data column (+ int)")
        self.patterns.append(Pattern("aug", Expr.lift(expr), data, name, target=con,
                                     row_col=row.name, row_off=row.shift))
        return len(self.patterns) - 1

    # -- flat arrays ----------------------------------------------------------
    @property
    def xl(self): return _cat(self._xl)
    @property
    def xu(self): return _cat(self._xu)
    @property
    def x0(self): return _cat(self._x0)
    @property
    def theta(self): return _cat(self._theta)

    def set_theta(self, theta):
        t = np.asarray(theta, dtype=np.float64).reshape(-1)
        if t.size != self.ntheta:
            raise ValueError("theta has the wrong length")
        self._theta = [t.copy()]

    @property
    def ncon(self) -> int:
        return sum(p.ndata for p in self.patterns if p.kind == "con")

    def con_offsets(self) -> Dict[int, int]:
        """First row of every base constraint block, in declaration order."""
        off, r = {}, 0
        for i, p in enumerate(self.patterns):
            if p.kind == "con":
                off[i] = r
                r += p.ndata
        return off

    @property
    def lcon(self):
        return _cat([p.lcon for p in self.patterns if p.kind == "con"])

    @property
    def ucon(self):
        return _cat([p.ucon for p in self.patterns if p.kind == "con"])


def _cat(xs):
    if not xs:
        return np.zeros(0, dtype=np.float64)
    return np.ascontiguousarray(np.concatenate(xs).astype(np.float64))
