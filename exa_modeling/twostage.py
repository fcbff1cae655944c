"""Two-stage stochastic layout (eq. extensions with one batch instance;
Sec. 7.4.2, two-stage stochastic programs).

Root (first-stage) blocks are declared once; scenario blocks are replicated
for S scenarios with the scenario index as the last dimension (entry j of
scenario s, 0-based, sits at j + n*s of its block).  Every variable and
constraint row is tagged with the scenario it belongs to: 0 for the root,
1..S for the scenarios.  The result is an ordinary :class:`Model`: the
scenarios are one more data dimension of the same patterns, so each pattern
is compiled once, and a root variable that every scenario touches becomes
one long reduction segment in the evaluator.  As with the rest of this
package, nothing here evaluates the model.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .ir import DataSet, Model, ParBlock, VarBlock


class TwoStageModel(Model):
    def __init__(self, nscen: int, name: str = "twostage"):
        if int(nscen) < 1:
            raise ValueError("a two-stage model needs at least one scenario")
        super().__init__(name)
        self.nscen = int(nscen)
        self._vtag: List[np.ndarray] = []
        self._ctag: List[np.ndarray] = []

    def _scen_tags(self, n: int) -> np.ndarray:
        return np.repeat(np.arange(1, self.nscen + 1, dtype=np.int64), n)

    def add_var(self, n: int, lvar=-math.inf, uvar=math.inf, start=0.0, name="", *,
                each_scenario: bool = False) -> VarBlock:
        """A root block of n variables, or with each_scenario a block of n
        variables per scenario (bounds and start given per entry j apply to
        every scenario)."""
        n = int(n)
        if not each_scenario:
            self._vtag.append(np.zeros(n, dtype=np.int64))
            return super().add_var(n, lvar, uvar, start, name)
        S = self.nscen
        rep = lambda a: np.tile(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)), S)  # noqa: E731
        self._vtag.append(self._scen_tags(n))
        return super().add_var(n * S, rep(lvar), rep(uvar), rep(start), name)

    def add_par(self, values, name="", *, each_scenario: bool = False) -> ParBlock:
        """Parameters: a root vector, or with each_scenario an (n, S) array
        whose column s holds scenario s's values."""
        if not each_scenario:
            return super().add_par(values, name)
        v = np.asarray(values, dtype=np.float64)
        if v.ndim != 2 or v.shape[1] != self.nscen:
            raise ValueError("scenario parameters must have shape (n, nscen)")
        return super().add_par(np.ascontiguousarray(v.T).reshape(-1), name)

    def add_con(self, expr, data: DataSet, lcon=0.0, ucon=0.0, name="", *,
                scenario: Optional[str] = None) -> int:
        """Constraint rows, one per data point; `scenario` names the integer
        data column holding each row's scenario (1..S), or None for root
        rows."""
        if scenario is None:
            tags = np.zeros(data.ndata, dtype=np.int64)
        else:
            if scenario not in data.icols:
                raise ValueError(f"no integer data column {scenario!r}")
            tags = np.asarray(data.icols[scenario], dtype=np.int64)
            if tags.size and (tags.min() < 1 or tags.max() > self.nscen):
                raise ValueError("scenario tags must lie in 1..nscen")
        self._ctag.append(tags)
        return super().add_con(expr, data, lcon, ucon, name)

    def var_scenario(self) -> np.ndarray:
        """Scenario of every variable (0 = root)."""
        return np.concatenate(self._vtag) if self._vtag else np.zeros(0, dtype=np.int64)

    def con_scenario(self) -> np.ndarray:
        """Scenario of every constraint row (0 = root)."""
        return np.concatenate(self._ctag) if self._ctag else np.zeros(0, dtype=np.int64)
