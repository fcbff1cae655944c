"""Two-stage stochastic layout (Sec. 7.4.2): block layout and scenario tags
on the host, and (GPU) every callback against the oracle on a model whose
root variables are shared by every scenario (long reduction segments)."""
import numpy as np
import pytest

from exa_modeling import DataSet, TwoStageModel
from exa_modeling.generators import two_stage
from oracle import OracleModel


def test_layout_and_tags():
    S, n0, nz = 5, 3, 4
    w = two_stage(S, n0, nz, seed=3)
    m = w.model
    assert m.nvar == n0 + nz * S and m.ncon == n0 + nz * S
    vs, cs = m.var_scenario(), m.con_scenario()
    assert vs.tolist() == [0] * n0 + [s for s in range(1, S + 1) for _ in range(nz)]
    assert cs.tolist() == [0] * n0 + [s for s in range(1, S + 1) for _ in range(nz)]
    # a row touches the root and its own scenario only
    o = OracleModel(m)
    rows, cols = o.jac_structure()
    for r, c in zip(rows, cols):
        assert vs[c] in (0, cs[r]), (r, c)
    hr, hc = o.hess_structure()
    for a, b in zip(hr, hc):
        assert vs[a] == 0 or vs[b] == 0 or vs[a] == vs[b]


def test_scenario_parameters_and_bounds():
    m = TwoStageModel(3)
    z = m.add_var(2, lvar=[-1.0, -2.0], uvar=[1.0, 2.0], name="z", each_scenario=True)
    vals = np.arange(6.0).reshape(2, 3)  # column s = scenario s
    d = m.add_par(vals, each_scenario=True)
    assert (z.offset, z.length) == (0, 6) and (d.offset, d.length) == (0, 6)
    assert m.theta.tolist() == [0.0, 3.0, 1.0, 4.0, 2.0, 5.0]  # entry j of scenario s at j + 2 s
    assert m.xl.tolist() == [-1.0, -2.0] * 3 and m.xu.tolist() == [1.0, 2.0] * 3
    data = DataSet(6, k=np.arange(6), scen=np.repeat([1, 2, 3], 2))
    m.add_con(z[data.k] * 2.0, data, scenario="scen")
    assert m.con_scenario().tolist() == [1, 1, 2, 2, 3, 3]
    with pytest.raises(ValueError):
        m.add_par(np.zeros((2, 2)), each_scenario=True)
    with pytest.raises(ValueError):
        m.add_con(z[data.k], DataSet(6, k=np.arange(6), scen=np.full(6, 4)), scenario="scen")
    with pytest.raises(ValueError):
        TwoStageModel(0)


def test_host_structure_matches_oracle():
    from paper_2608_16265_amd import ExaModel
    w = two_stage(40, 4, 8, seed=2)
    em = ExaModel(w.model, host_only=True)
    o = OracleModel(w.model)
    for g, r in zip(em.jac_structure(), o.jac_structure()):
        assert np.array_equal(g, r)
    for g, r in zip(em.hess_structure(), o.hess_structure()):
        assert np.array_equal(g, r)
