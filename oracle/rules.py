"""Simplification and sparsity structure of one pattern (oracle side).

Test infrastructure: see the package docstring.

* :func:`simplify` applies the identities of Sec. 7.1.2 bottom-up.
* :func:`first_order_visits` lists the variable leaves in the order the
  first-order reverse pass reaches them (Sec. 5.2.1 probe): a left-to-right
  depth-first walk, first child before second child.
* :func:`second_order_visits` lists the (a, b) variable pairs in the order a
  second-order reverse pass emits them, under the reading that a second
  adjoint is structurally zero until some ancestor with curvature is met
  (Sec. 5.1.3 hrpass/hdrpass, Sec. 7.2.2 affine nodes).
* :func:`compress` turns a visit list into the unique list and the
  ``comp`` map of Sec. 5.2.2 (1-based, as printed in the paper).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Tuple


@dataclass
class T:
    """A tree node held by the oracle."""
    op: str
    args: tuple = ()
    value: float = 0.0
    col: Optional[str] = None
    off: int = 0

    def key(self):
        """Symbolic identity of a var/param reference (index column, offset)."""
        return (self.op, self.col, self.off)


def from_nodes(nodes) -> T:
    """Rebuild a tree from the post-order node list of the model description."""
    built: List[T] = []
    for n in nodes:
        if n.op in ("const", "data", "var", "param"):
            built.append(T(n.op, (), n.value, n.col, n.off))
        elif n.b < 0:
            built.append(T(n.op, (built[n.a],)))
        else:
            built.append(T(n.op, (built[n.a], built[n.b])))
    return built[-1]


def _is_const(t: T, v: float) -> bool:
    return t.op == "const" and t.value == v


def simplify(t: T) -> T:
    """Apply the Sec. 7.1.2 table bottom-up.

    x+0 -> x (either side), x*1 -> x (either side), x/1 -> x, x^0 -> 1,
    x^1 -> x, x^2 -> abs2(x), x^-1 -> inv(x), 0*x -> 0 (either side),
    0/x -> 0.  Only literal constants trigger a rule; nothing else is folded.
    """
    if not t.args:
        return t
    a = tuple(simplify(c) for c in t.args)
    op = t.op
    if op == "add":
        if _is_const(a[1], 0.0):
            return a[0]
        if _is_const(a[0], 0.0):
            return a[1]
    elif op == "mul":
        if _is_const(a[0], 0.0) or _is_const(a[1], 0.0):
            return T("const", value=0.0)
        if _is_const(a[1], 1.0):
            return a[0]
        if _is_const(a[0], 1.0):
            return a[1]
    elif op == "div":
        if _is_const(a[0], 0.0):
            return T("const", value=0.0)
        if _is_const(a[1], 1.0):
            return a[0]
    elif op == "pow" and a[1].op == "const":
        e = a[1].value
        if e == 0.0:
            return T("const", value=1.0)
        if e == 1.0:
            return a[0]
        if e == 2.0:
            return T("abs2", (a[0],))
        if e == -1.0:
            return T("inv", (a[0],))
    return T(op, a)


def has_var(t: T) -> bool:
    if t.op == "var":
        return True
    return any(has_var(c) for c in t.args)


def var_leaves(t: T) -> List[T]:
    """Variable leaves in left-to-right depth-first order."""
    if t.op == "var":
        return [t]
    out: List[T] = []
    for c in t.args:
        out += var_leaves(c)
    return out


def param_leaves(t: T) -> List[T]:
    if t.op == "param":
        return [t]
    out: List[T] = []
    for c in t.args:
        out += param_leaves(c)
    return out


def first_order_visits(t: T) -> List[tuple]:
    """Symbolic var references in first-order reverse-pass order (Sec. 5.2.1)."""
    return [v.key() for v in var_leaves(t)]


# Curvature of each operator, used by the second-order emission rule.
# Unary: does F'' vanish identically?
_UNARY_AFFINE = {"neg"}
# Binary with variables on both sides: (F11 nonzero, F12 nonzero, F22 nonzero).
_BINARY_CURV = {
    "add": (False, False, False),
    "sub": (False, False, False),
    "mul": (False, True, False),
    "div": (False, True, True),
    "pow": (True, True, True),
}


def _one_sided_affine(op: str, var_on_left: bool) -> bool:
    """Binary node with one variable-free side, seen as a unary map of the
    other side: is it affine in that side?  (Sec. 7.2.2 FirstFixed/SecondFixed.)"""
    if op in ("add", "sub", "mul"):
        return True
    if op == "div":
        return var_on_left          # u / c is affine, c / u is not
    return False                    # u^c and c^u


def second_order_visits(t: T) -> List[Tuple[tuple, tuple]]:
    """(a, b) var pairs in second-order reverse-pass emission order.

    Rule, with ``nl`` = "some ancestor's curvature reaches this node"
    (false at the root):
      var leaf: emit (v, v) when nl;
      const/data/param: nothing;
      unary F(u): recurse into u with nl or (F not affine);
      binary with one variable-free side: as a unary map of the other side;
      binary F(u, w) with variables on both sides: recurse into u with
      nl or F11, then into w with nl or F22, then, when nl or F12, emit
      every pair (leaf of u, leaf of w) in depth-first order.
    """
    out: List[Tuple[tuple, tuple]] = []

    def H(node: T, nl: bool):
        if node.op == "var":
            if nl:
                out.append((node.key(), node.key()))
            return
        if not node.args:
            return
        if len(node.args) == 1:
            H(node.args[0], nl or node.op not in _UNARY_AFFINE)
            return
        u, w = node.args
        hu, hw = has_var(u), has_var(w)
        if hu and hw:
            f11, f12, f22 = _BINARY_CURV[node.op]
            H(u, nl or f11)
            H(w, nl or f22)
            if nl or f12:
                for lu in var_leaves(u):
                    for lw in var_leaves(w):
                        out.append((lu.key(), lw.key()))
        elif hu:
            H(u, nl or not _one_sided_affine(node.op, True))
        elif hw:
            H(w, nl or not _one_sided_affine(node.op, False))

    H(t, False)
    return out


def compress(raw: list, pairs: bool = False):
    """Unique entries of a visit list and the 1-based map from visit to entry.

    For pairs the entry is unordered: (a, b) and (b, a) are the same slot.
    """
    uniq: list = []
    keys: list = []
    comp: List[int] = []
    for r in raw:
        k = frozenset(r) if pairs else r
        if k not in keys:
            keys.append(k)
            uniq.append(r)
        comp.append(keys.index(k) + 1)
    return uniq, comp
