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


def test_dropped_row_offset_is_caught(monkeypatch):
    """An augmentation row without its offset (icol[k] instead of
    icol[k] + row_off) must fail the closed-form pin."""
    from oracle.nlp import OracleModel
    from test_oracle_pins import aug_offset_case
    from oracle_checks import check_aug_offset

    def rows_without_offset(self, P, ks):
        if P.kind == "con":
            return P.o0 + ks
        return P.target_o0 + P.icols[P.row_col][ks].astype(np.int64)
    assert check_aug_offset(aug_offset_case()) < 1e-15
    monkeypatch.setattr(OracleModel, "_rows", rows_without_offset)
    assert check_aug_offset(aug_offset_case()) > 1e-3


@pytest.mark.parametrize("kind", ["neighbour_row", "sigma_for_all", "no_weight"])
def test_hessian_weight_mistake_is_caught(monkeypatch, kind):
    """A wrong Hessian weight in hess_block (y of another row, sigma for a
    constraint, no weight at all) must fail a closed-form pin."""
    from oracle.nlp import OracleModel
    from test_oracle_pins import aug_offset_case
    from oracle_checks import check_aug_offset
    orig = OracleModel._weights

    def bad(self, P, ks, y, sigma, dtype=np.float64):
        w = orig(self, P, ks, y, sigma, dtype)
        if P.kind == "obj":
            return w
        if kind == "neighbour_row":
            return np.asarray(y, dtype=dtype)[(self._rows(P, ks) + 1) % len(y)]
        if kind == "sigma_for_all":
            return np.full(ks.size, sigma, dtype=dtype)
        return np.ones(ks.size, dtype=dtype)
    monkeypatch.setattr(OracleModel, "_weights", bad)
    assert check_aug_offset(aug_offset_case()) > 1e-3


def test_dropped_alias_doubling_is_caught(monkeypatch):
    """hess_block without the doubling of a cross pair that resolves to a
    diagonal position must fail the aliasing pin (duplicates summing to the
    true Hessian)."""
    import test_oracle_pins
    from oracle.nlp import OracleModel

    def no_doubling(self, i, ks, x, y, sigma=1.0, theta=None, dtype=np.float64):
        P = self.pats[i]
        ks = np.asarray(ks, dtype=np.int64)
        t = self._taylor(P, ks, x, self._theta(theta), dtype=dtype)
        w = self._weights(P, ks, y, sigma, dtype)
        return np.stack([w * t.h[:, a, b] for a, b in P.hslots], axis=1) if P.hslots else \
            np.zeros((ks.size, 0), dtype=dtype)
    monkeypatch.setattr(OracleModel, "hess_block", no_doubling)
    with pytest.raises(AssertionError):
        test_oracle_pins.test_aliased_references_sum_to_true_hessian()
