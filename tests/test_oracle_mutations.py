"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins of test_oracle_pins.py would catch each of them."""
import numpy as np
import pytest

from exa_modeling.generators import acopf
from oracle import rules, taylor
from oracle_checks import check_coverage, check_first_order, check_second_order
from test_oracle_pins import op_zoo


def _mutate_unary(monkeypatch, op, which, fn):
    orig = taylor.unary_derivs

    def mutated(o, u):
        out = list(orig(o, u))
        if o == op:
            out[which] = fn(u, out[which])
        return tuple(out)
    monkeypatch.setattr(taylor, "unary_derivs", mutated)


def _mutate_binary(monkeypatch, op, which, fn):
    orig = taylor.binary_derivs

    def mutated(o, u, w, uc, wc):
        out = list(orig(o, u, w, uc, wc))
        if o == op:
            out[which] = fn(u, w, out[which])
        return tuple(out)
    monkeypatch.setattr(taylor, "binary_derivs", mutated)


FIRST = [  # mistakes in a first derivative: complex step must catch them
    ("sin'", lambda mp: _mutate_unary(mp, "sin", 1, lambda u, d: -d)),
    ("exp'", lambda mp: _mutate_unary(mp, "exp", 1, lambda u, d: d * 1.0000001)),
    ("div F2 sign", lambda mp: _mutate_binary(mp, "div", 2, lambda u, w, d: -d)),
    ("mul operands swapped", lambda mp: _mutate_binary(mp, "mul", 1, lambda u, w, d: u)),
    ("pow F1", lambda mp: _mutate_binary(mp, "pow", 1, lambda u, w, d: d * w)),
    ("atan'", lambda mp: _mutate_unary(mp, "atan", 1, lambda u, d: 1.0 / (1.0 - u * u))),
]
SECOND = [  # mistakes in a second derivative: FD of the gradient must catch them
    ("cos''", lambda mp: _mutate_unary(mp, "cos", 2, lambda u, d: -d)),
    ("abs2''", lambda mp: _mutate_unary(mp, "abs2", 2, lambda u, d: d * 0.5)),
    ("mul F12 dropped", lambda mp: _mutate_binary(mp, "mul", 4, lambda u, w, d: 0 * d)),
    ("div F22 dropped", lambda mp: _mutate_binary(mp, "div", 5, lambda u, w, d: 0 * d)),
    ("tanh''", lambda mp: _mutate_unary(mp, "tanh", 2, lambda u, d: 0 * d)),
]


@pytest.mark.parametrize("name,plant", FIRST, ids=[n for n, _ in FIRST])
def test_first_order_mistake_is_caught(monkeypatch, name, plant):
    plant(monkeypatch)
    assert check_first_order(op_zoo()) > 1e-8 or check_first_order(acopf(30, 0)) > 1e-8


@pytest.mark.parametrize("name,plant", SECOND, ids=[n for n, _ in SECOND])
def test_second_order_mistake_is_caught(monkeypatch, name, plant):
    plant(monkeypatch)
    assert max(check_second_order(op_zoo()), check_second_order(acopf(30, 0))) > 1e-4


def test_dropped_chain_rule_term_is_caught(monkeypatch):
    orig_outer = taylor._outer
    calls = {"n": 0}

    def bad_outer(a, b):  # drop the first outer-product term of every node
        calls["n"] += 1
        return orig_outer(a, b) * (0.0 if calls["n"] % 3 == 1 else 1.0)
    monkeypatch.setattr(taylor, "_outer", bad_outer)
    assert max(check_second_order(op_zoo()), check_second_order(acopf(30, 0))) > 1e-4


def test_missing_cross_pairs_are_caught(monkeypatch):
    orig = rules._BINARY_CURV.copy()
    monkeypatch.setitem(rules._BINARY_CURV, "mul", (False, False, False))
    assert check_coverage(acopf(30, 0)) > 0.0
    monkeypatch.setattr(rules, "_BINARY_CURV", orig)


def test_wrong_linear_classification_is_caught(monkeypatch):
    monkeypatch.setattr(rules, "_UNARY_AFFINE", {"neg", "sin", "cos"})
    assert check_coverage(acopf(30, 0)) > 0.0
