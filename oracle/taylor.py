"""Second-order forward mode over a pattern tree (oracle side).

Test infrastructure: see the package docstring.

A :class:`Taylor` value holds, for every data point of a pattern, the value
v of a node, its gradient g (length m) and its Hessian h (m x m) with
respect to m local independents (the pattern's unique variable references,
optionally followed by its unique parameter references).  Each operator
maps children to parent with the chain rule

  unary   y = F(u):   g = F' gu,  h = F' hu + F'' gu gu^T
  binary  y = F(u,w): g = F1 gu + F2 gw,
                      h = F1 hu + F2 hw + F11 gu gu^T
                          + F12 (gu gw^T + gw gu^T) + F22 gw gw^T

with the operator's own first and second derivatives (the registration
triple f, f', f'' of Sec. 7.1.3).  Arrays are vectorised over data points
and work with float64 or complex128 (the latter for complex-step checks).
"""
from __future__ import annotations

import numpy as np


class Taylor:
    __slots__ = ("v", "g", "h")

    def __init__(self, v, g, h):
        self.v, self.g, self.h = v, g, h


def _outer(a, b):
    return a[:, :, None] * b[:, None, :]


# unary: name -> (F, F', F'') as functions of u
def _unary_table(u):
    return {
        "neg":   lambda: (-u, -np.ones_like(u), np.zeros_like(u)),
        "abs2":  lambda: (u * u, 2.0 * u, 2.0 * np.ones_like(u)),
        "inv":   lambda: (1.0 / u, -1.0 / (u * u), 2.0 / (u * u * u)),
        "sqrt":  lambda: (np.sqrt(u), 0.5 / np.sqrt(u), -0.25 / (u * np.sqrt(u))),
        "exp":   lambda: (np.exp(u), np.exp(u), np.exp(u)),
        "log":   lambda: (np.log(u), 1.0 / u, -1.0 / (u * u)),
        "sin":   lambda: (np.sin(u), np.cos(u), -np.sin(u)),
        "cos":   lambda: (np.cos(u), -np.sin(u), -np.cos(u)),
        "tan":   lambda: (np.tan(u), 1.0 / np.cos(u) ** 2,
                          2.0 * np.tan(u) / np.cos(u) ** 2),
        "atan":  lambda: (np.arctan(u), 1.0 / (1.0 + u * u),
                          -2.0 * u / (1.0 + u * u) ** 2),
        "sinh":  lambda: (np.sinh(u), np.cosh(u), np.sinh(u)),
        "cosh":  lambda: (np.cosh(u), np.sinh(u), np.cosh(u)),
        "tanh":  lambda: (np.tanh(u), 1.0 / np.cosh(u) ** 2,
                          -2.0 * np.tanh(u) / np.cosh(u) ** 2),
        "log1p": lambda: (np.log1p(u), 1.0 / (1.0 + u), -1.0 / (1.0 + u) ** 2),
        "expm1": lambda: (np.expm1(u), np.exp(u), np.exp(u)),
    }


def unary_derivs(op, u):
    tab = _unary_table(u)
    if op not in tab:
        raise ValueError(f"oracle: unknown unary operator {op!r}")
    return tab[op]()


def binary_derivs(op, u, w, u_const: bool, w_const: bool):
    """(F, F1, F2, F11, F12, F22).  ``*_const`` says a side carries no
    independent, so the derivative terms in it are not formed (this keeps
    log(u) out of u^c for negative u)."""
    one, zero = np.ones_like(u * w), np.zeros_like(u * w)
    if op == "add":
        return u + w, one, one, zero, zero, zero
    if op == "sub":
        return u - w, one, -one, zero, zero, zero
    if op == "mul":
        return u * w, w * one, u * one, zero, one, zero
    if op == "div":
        return u / w, 1.0 / w * one, -u / (w * w), zero, -1.0 / (w * w) * one, 2.0 * u / (w * w * w)
    if op == "pow":
        F = u ** w
        if w_const:
            return F, w * u ** (w - 1.0), zero, w * (w - 1.0) * u ** (w - 2.0), zero, zero
        lu = np.log(u)
        if u_const:
            return F, zero, F * lu, zero, zero, F * lu * lu
        return (F, w * u ** (w - 1.0), F * lu, w * (w - 1.0) * u ** (w - 2.0),
                u ** (w - 1.0) * (1.0 + w * lu), F * lu * lu)
    raise ValueError(f"oracle: unknown binary operator {op!r}")


def evaluate(t, leaf, m: int, npts: int, dtype=np.float64) -> Taylor:
    """Evaluate tree ``t`` on ``npts`` data points.

    ``leaf(node)`` returns (value array, independent position or -1) for
    var/param/data/const leaves; positions index the m local independents.
    Returns the Taylor value of the root.
    """
    def zeros_g():
        return np.zeros((npts, m), dtype=dtype)

    def zeros_h():
        return np.zeros((npts, m, m), dtype=dtype)

    def rec(node):
        if not node.args:
            val, pos = leaf(node)
            val = np.broadcast_to(np.asarray(val, dtype=dtype), (npts,)).copy()
            g = zeros_g()
            if pos >= 0:
                g[:, pos] = 1.0
            return Taylor(val, g, zeros_h()), pos < 0
        if len(node.args) == 1:
            u, _ = rec(node.args[0])
            F, F1, F2 = unary_derivs(node.op, u.v)
            g = F1[:, None] * u.g
            h = F1[:, None, None] * u.h + F2[:, None, None] * _outer(u.g, u.g)
            return Taylor(F, g, h), _
        (u, uc), (w, wc) = rec(node.args[0]), rec(node.args[1])
        F, F1, F2, F11, F12, F22 = binary_derivs(node.op, u.v, w.v, uc, wc)
        g = F1[:, None] * u.g + F2[:, None] * w.g
        h = (F1[:, None, None] * u.h + F2[:, None, None] * w.h
             + F11[:, None, None] * _outer(u.g, u.g)
             + F12[:, None, None] * (_outer(u.g, w.g) + _outer(w.g, u.g))
             + F22[:, None, None] * _outer(w.g, w.g))
        return Taylor(F, g, h), uc and wc

    return rec(t)[0]


def evaluate_value(t, leaf, npts: int, dtype=np.float64):
    """Value only (zeroth order), for objective/constraint values and the
    complex-step checks."""
    def rec(node):
        if not node.args:
            val, _ = leaf(node)
            return np.broadcast_to(np.asarray(val, dtype=dtype), (npts,))
        if len(node.args) == 1:
            return unary_derivs(node.op, rec(node.args[0]))[0]
        u, w = rec(node.args[0]), rec(node.args[1])
        return binary_derivs(node.op, u, w, True, True)[0]
    return rec(t)
