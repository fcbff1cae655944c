"""Seeded synthetic workloads shaped like the paper's benchmark families.

The paper measures on PGLib-OPF power-flow cases, on COPS and on the
Luksan-Vlcek set (Sec. 8.1).  None of those files is available here, so
these generators draw synthetic instances with the same algebraic patterns
and comparable sizes; they stand in for those suites and are not copies of
any of their instances.

* :func:`acopf` -- AC optimal power flow in polar form, built in the layered
  way of Sec. 3.3.2 (base balance rows plus augmentations), 13 patterns.
* :func:`pde` -- distributed control of a semilinear elliptic PDE on an
  n x n grid (5-point Laplacian), a COPS-like shape.
* :func:`rosenbrock` -- the extended Rosenbrock objective, eq. rosenbrock.
* :func:`goddard` -- the Goddard rocket, eq. rocket, with the constants of
  the modeling example of Sec. 2.2.2.
* :func:`kernel_sweep` -- k of sixteen two-variable constraint patterns over
  a fixed number of rows (the compilation study of Sec. 8.6).
* :func:`two_stage` -- a two-stage stochastic model (Sec. 7.4.2): a few root
  variables shared by every scenario, replicated scenario blocks.

Every random draw comes from ``numpy.random.Generator(PCG64(seed))`` in a
fixed order, documented per function.  Nothing here evaluates the model.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict

import numpy as np

from .ir import (DataSet, Model, abs2, atan, cos, cosh, exp, expm1, log1p, sin, sinh, sqrt, tanh)


@dataclass
class Workload:
    """A model plus one evaluation point (x, y, sigma) drawn with it."""
    model: Model
    x: np.ndarray
    y: np.ndarray
    sigma: float = 1.0
    meta: Dict = field(default_factory=dict)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def acopf_topology(rng: np.random.Generator, nb: int):
    """Ring over the buses plus ``ceil(0.35 nb)`` random chords.

    Chords are drawn as (from, to) pairs uniformly over the buses and
    rejected when they are self-loops or repeat an existing branch in either
    direction.  Returns (fr, to) int arrays of length nl.
    """
    nc = (35 * nb + 99) // 100
    fr = list(range(nb))
    to = [(i + 1) % nb for i in range(nb)]
    seen = set()
    for a, b in zip(fr, to):
        seen.add((min(a, b), max(a, b)))
    cf, ct = [], []
    while len(cf) < nc:
        need = nc - len(cf)
        cand = rng.integers(0, nb, size=(2 * need + 8, 2))
        for a, b in cand:
            a, b = int(a), int(b)
            key = (min(a, b), max(a, b))
            if a == b or key in seen:
                continue
            seen.add(key)
            cf.append(a)
            ct.append(b)
            if len(cf) == nc:
                break
    return (np.asarray(fr + cf, dtype=np.int64), np.asarray(to + ct, dtype=np.int64))


def acopf(nb: int, seed: int, *, load_perturb: bool = False, gb_in_theta: bool = False,
          rng: np.random.Generator = None) -> Workload:
    """ACOPF-shaped NLP in polar form with ``nb`` buses.

    Draw order: topology (ring, chords), generator buses, g, b, rate, pd, qd,
    c0, c1, c2, then the point x (va, vm, pg, qg, p, q), then y; with
    ``load_perturb`` one factor U(0.9, 1.1) per bus is drawn last and scales
    pd and qd.

    Variables: va[nb], vm[nb], pg[ng], qg[ng], p[2 nl], q[2 nl] where arc
    ``l`` (0 <= l < nl) is the from end of branch l and arc ``nl + l`` its to
    end.  Parameters theta = (pd[nb], qd[nb], c1[ng], c2[ng]) and, with
    ``gb_in_theta``, also (g[nl], b[nl]).

    Patterns, in declaration order:
      0 O    sum over generators of c2 pg^2 + c1 pg + c0
      1 C_pf p_f - (g vm_f^2 - vm_f vm_t (g cos(va_f - va_t) + b sin(va_f - va_t)))
      2 C_qf q_f - (-b vm_f^2 - vm_f vm_t (g sin(va_f - va_t) - b cos(va_f - va_t)))
      3 C_pt, 4 C_qt   the same at the to end (f and t swapped)
      5 B_p  pd_b  (one row per bus)       6 B_q  qd_b
      7 A_pg B_p[bus(g)] += -pg_g          8 A_qg B_q[bus(g)] += -qg_g
      9 A_p  B_p[bus(a)] += p_a            10 A_q B_q[bus(a)] += q_a
      11 T_f p_f^2 + q_f^2 <= rate^2       12 T_t p_t^2 + q_t^2 <= rate^2
    """
    if rng is None:
        rng = _rng(seed)
    nb = int(nb)
    fr, to = acopf_topology(rng, nb)
    nl = fr.size
    ng = (nb + 2) // 5
    gen_bus = rng.choice(nb, size=ng, replace=False).astype(np.int64)
    g = rng.uniform(1.0, 10.0, nl)
    b = rng.uniform(-20.0, -5.0, nl)
    rate = rng.uniform(0.5, 5.0, nl)
    pd = rng.uniform(0.0, 1.0, nb)
    qd = rng.uniform(0.0, 1.0, nb)
    c0 = rng.uniform(0.0, 1.0, ng)
    c1 = rng.uniform(10.0, 40.0, ng)
    c2 = rng.uniform(0.01, 0.1, ng)
    va0 = rng.uniform(-0.3, 0.3, nb)
    vm0 = rng.uniform(0.9, 1.1, nb)
    pg0 = rng.uniform(0.0, 2.0, ng)
    qg0 = rng.uniform(-1.0, 1.0, ng)
    p0 = rng.uniform(-1.0, 1.0, 2 * nl)
    q0 = rng.uniform(-1.0, 1.0, 2 * nl)
    m_rows = 6 * nl + 2 * nb
    y = rng.standard_normal(m_rows)
    if load_perturb:
        fac = rng.uniform(0.9, 1.1, nb)
        pd = pd * fac
        qd = qd * fac

    m = Model(f"acopf{nb}")
    va = m.add_var(nb, name="va", start=0.0)
    vm = m.add_var(nb, lvar=0.9, uvar=1.1, start=1.0, name="vm")
    pg = m.add_var(ng, lvar=0.0, uvar=2.0, name="pg")
    qg = m.add_var(ng, lvar=-1.0, uvar=1.0, name="qg")
    p = m.add_var(2 * nl, name="p")
    q = m.add_var(2 * nl, name="q")
    th_pd = m.add_par(pd, "pd")
    th_qd = m.add_par(qd, "qd")
    th_c1 = m.add_par(c1, "c1")
    th_c2 = m.add_par(c2, "c2")

    gens = DataSet(ng, i=np.arange(ng), bus=gen_bus, c0=c0)
    m.add_obj(th_c2[gens.i] * pg[gens.i] ** 2 + th_c1[gens.i] * pg[gens.i] + gens.c0, gens, "O")

    br = DataSet(nl, l=np.arange(nl), f=fr, t=to, g=g, b=b)
    if gb_in_theta:
        th_g = m.add_par(g, "g")
        th_b = m.add_par(b, "b")
        G, B = th_g[br.l], th_b[br.l]
    else:
        G, B = br.g, br.b

    def flow_p(pi, vi, vj, ai, aj):
        return pi - (G * vi ** 2 - vi * vj * (G * cos(ai - aj) + B * sin(ai - aj)))

    def flow_q(qi, vi, vj, ai, aj):
        return qi - (-B * vi ** 2 - vi * vj * (G * sin(ai - aj) - B * cos(ai - aj)))

    vf, vt, af, at = vm[br.f], vm[br.t], va[br.f], va[br.t]
    m.add_con(flow_p(p[br.l], vm[br.f], vm[br.t], va[br.f], va[br.t]), br, name="C_pf")
    m.add_con(flow_q(q[br.l], vm[br.f], vm[br.t], va[br.f], va[br.t]), br, name="C_qf")
    m.add_con(flow_p(p[br.l + nl], vm[br.t], vm[br.f], va[br.t], va[br.f]), br, name="C_pt")
    m.add_con(flow_q(q[br.l + nl], vm[br.t], vm[br.f], va[br.t], va[br.f]), br, name="C_qt")
    del vf, vt, af, at

    buses = DataSet(nb, b=np.arange(nb))
    bp = m.add_con(th_pd[buses.b], buses, name="B_p")
    bq = m.add_con(th_qd[buses.b], buses, name="B_q")
    m.add_con_aug(bp, gens.bus, -pg[gens.i], gens, name="A_pg")
    m.add_con_aug(bq, gens.bus, -qg[gens.i], gens, name="A_qg")
    arcs = DataSet(2 * nl, a=np.arange(2 * nl), bus=np.concatenate([fr, to]))
    m.add_con_aug(bp, arcs.bus, p[arcs.a], arcs, name="A_p")
    m.add_con_aug(bq, arcs.bus, q[arcs.a], arcs, name="A_q")
    m.add_con(p[br.l] ** 2 + q[br.l] ** 2, br, lcon=-np.inf, ucon=rate ** 2, name="T_f")
    m.add_con(p[br.l + nl] ** 2 + q[br.l + nl] ** 2, br, lcon=-np.inf, ucon=rate ** 2, name="T_t")

    x = np.concatenate([va0, vm0, pg0, qg0, p0, q0])
    assert x.size == m.nvar and m.ncon == m_rows
    meta = dict(nb=nb, nl=nl, ng=ng, seed=seed, fr=fr, to=to, gen_bus=gen_bus,
                offsets=dict(va=va.offset, vm=vm.offset, pg=pg.offset, qg=qg.offset,
                             p=p.offset, q=q.offset),
                theta_offsets=dict(pd=th_pd.offset, qd=th_qd.offset, c1=th_c1.offset,
                                   c2=th_c2.offset))
    return Workload(m, x, y, 1.0, meta)


def acopf_batch_sizes(count: int, first_seed: int, lo: int = 500, hi: int = 20000):
    """Bus counts log-uniform in [lo, hi], one generator per instance seed.

    Instance ``i`` uses seed ``first_seed + i``; its first draw is the bus
    count ``round(exp(U(ln lo, ln hi)))``, after which :func:`acopf` continues
    on the same generator.
    """
    out = []
    for i in range(count):
        rng = _rng(first_seed + i)
        nb = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append((first_seed + i, nb, rng))
    return out


def acopf_batch(count: int = 256, first_seed: int = 1000, lo: int = 500, hi: int = 20000):
    """The uneven batch of ACOPF instances with loads perturbed by U(0.9, 1.1)."""
    return [acopf(nb, seed, load_perturb=True, rng=rng)
            for seed, nb, rng in acopf_batch_sizes(count, first_seed, lo, hi)]


def acopf_batch_instance(seed: int, lo: int = 500, hi: int = 20000) -> Workload:
    """Instance ``seed - first_seed`` of :func:`acopf_batch`, drawn alone
    (each instance has a generator of its own)."""
    rng = _rng(seed)
    nb = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    return acopf(nb, seed, load_perturb=True, rng=rng)


def pde(n: int, seed: int) -> Workload:
    """Distributed control of -Laplace(u) + exp(u) = f on an n x n grid.

    h = 1/(n-1), grid point (i, j) at (i h, j h), linear index c = i n + j.
    Variables: u[n^2], f[n^2] (state and control).  Objective (no quadrature
    weights): sum 0.5 (u_c - ut_c)^2 + sum 1e-4 f_c^2 with
    ut = sin(pi x) sin(pi y).  One constraint per interior point:
    (4 u_c - u_{c-n} - u_{c+n} - u_{c+1} - u_{c-1}) / h^2 + exp(u_c) - f_c = 0.
    Bounds: u = 0 on the boundary, 0 <= f <= 10.

    Draw order: u = ut + 0.1 N(0, 1) (n^2 values), f ~ U(0, 10), y ~ N(0, 1).
    """
    rng = _rng(seed)
    n = int(n)
    if n < 3:
        raise ValueError("the grid needs n >= 3")
    N = n * n
    h = 1.0 / (n - 1)
    ih2 = float((n - 1) ** 2)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ut = (np.sin(math.pi * ii * h) * np.sin(math.pi * jj * h)).reshape(-1)
    boundary = ((ii == 0) | (ii == n - 1) | (jj == 0) | (jj == n - 1)).reshape(-1)
    interior = np.flatnonzero(~boundary)

    m = Model(f"pde{n}")
    ul = np.where(boundary, 0.0, -np.inf)
    uu = np.where(boundary, 0.0, np.inf)
    u = m.add_var(N, lvar=ul, uvar=uu, name="u")
    f = m.add_var(N, lvar=0.0, uvar=10.0, name="f")
    pts = DataSet(N, c=np.arange(N), ut=ut)
    m.add_obj(0.5 * (u[pts.c] - pts.ut) ** 2, pts, "O_u")
    m.add_obj(1e-4 * f[pts.c] ** 2, pts, "O_f")
    inn = DataSet(interior.size, c=interior)
    c = inn.c
    m.add_con((4 * u[c] - u[c - n] - u[c + n] - u[c + 1] - u[c - 1]) * ih2 + exp(u[c]) - f[c],
              inn, name="C_pde")

    u0 = ut + 0.1 * rng.standard_normal(N)
    f0 = rng.uniform(0.0, 10.0, N)
    y = rng.standard_normal(interior.size)
    x = np.concatenate([u0, f0])
    return Workload(m, x, y, 1.0, dict(n=n, interior=interior, h=h))


def rosenbrock(N: int, seed: int = 0) -> Workload:
    """Extended Rosenbrock, eq. rosenbrock, written as in Sec. 4.1.2.

    Data points i = 1 .. N-1 (0-based) with terms
    100 (x_{i-1}^2 - x_i)^2 + (x_{i-1} - 1)^2.  Point x ~ U(-2, 2).
    """
    rng = _rng(seed)
    m = Model(f"rosenbrock{N}")
    x = m.add_var(N, name="x")
    d = DataSet(N - 1, i=np.arange(1, N))
    i = d.i
    m.add_obj(100 * (x[i - 1] ** 2 - x[i]) ** 2 + (x[i - 1] - 1) ** 2, d, "rosen")
    x0 = rng.uniform(-2.0, 2.0, N)
    return Workload(m, x0, np.zeros(0), 1.0, dict(N=N))


def goddard(T: int, seed: int = 0) -> Workload:
    """Goddard rocket, eq. rocket (Sec. 1), trapezoidal rule over T steps,
    with the constants of the modeling example of Sec. 2.2.2.

    Variables h, v, m, tau over t = 0..T and the step dt (one entry, shared
    by every data point).  Constraint patterns over t = 1..T: altitude,
    velocity and mass dynamics; four singleton rows fix h_0, v_0, m_0 and
    m_T = m_f (m_f is a parameter).  Objective: maximise h_T, written as
    minimising -h_T.  Drag D(h, v) = D_c v^2 exp(-h_c (h - h0)/h0), gravity
    g(h) = g0 (h0/h)^2.  The point is the example's start point plus a
    seeded perturbation (so that no derivative is identically zero); y ~ N(0,1).
    """
    h0, v0, m0, g0 = 1.0, 0.0, 1.0, 1.0
    Tc, hc, vc, mc = 3.5, 500.0, 620.0, 0.6
    ce = 0.5 * math.sqrt(g0 * h0)
    mf = mc * m0
    Dc = 0.5 * vc * (m0 / g0)
    Tmax = Tc * m0 * g0
    rng = _rng(seed)
    m = Model(f"goddard{T}")
    h = m.add_var(T + 1, lvar=1.0, name="h")
    v = m.add_var(T + 1, name="v")
    ms = m.add_var(T + 1, lvar=mf, uvar=m0, name="m")
    tau = m.add_var(T + 1, lvar=0.0, uvar=Tmax, name="tau")
    dt = m.add_var(1, lvar=0.0, name="dt")
    th = m.add_par([mf], name="mf")
    d = DataSet(T, t=np.arange(1, T + 1))
    t = d.t

    def drag(hh, vv):
        return Dc * abs2(vv) * exp(-hc * (hh - h0) / h0)

    def grav(hh):
        return g0 * abs2(h0 / hh)

    m.add_con(h[t] - h[t - 1] - 0.5 * dt[0] * (v[t] + v[t - 1]), d, name="alt")
    m.add_con(v[t] - v[t - 1] - 0.5 * dt[0] * ((tau[t] - drag(h[t], v[t])) / ms[t] - grav(h[t])
                                                + (tau[t - 1] - drag(h[t - 1], v[t - 1])) / ms[t - 1]
                                                - grav(h[t - 1])), d, name="vel")
    m.add_con(ms[t] - ms[t - 1] + 0.5 * dt[0] / ce * (tau[t] + tau[t - 1]), d, name="mass")
    one = DataSet(1, k=np.zeros(1, dtype=np.int64))
    m.add_con(h[0] - h0, one, name="h0")
    m.add_con(v[0] - v0, one, name="v0")
    m.add_con(ms[0] - m0, one, name="m0")
    m.add_con(ms[T] - th[0], one, name="mT")
    m.add_obj(-h[T], one, name="hT")
    s = np.arange(T + 1) / T
    x = np.concatenate([1.0 + 0.01 * rng.uniform(0.0, 1.0, T + 1),
                        s * (1 - s) + 0.01 * rng.standard_normal(T + 1),
                        (mf - m0) * s + m0 + 0.01 * rng.uniform(0.0, 1.0, T + 1) * (m0 - mf),
                        Tmax / 2 + 0.1 * rng.standard_normal(T + 1),
                        [1.0 / T]])
    y = rng.standard_normal(m.ncon)
    return Workload(m, x, y, 1.0, dict(T=T))


def _sweep_patterns(a, b):
    """Sixteen distinct algebraic patterns over a variable pair (x_i, x_i+1)
    for the compilation-time study of Sec. 8.6 (the first five are the ones
    the paper names; the rest are of the same kind)."""
    return [a ** 2 + b, sin(a) * b, exp(a - b), sqrt(a ** 2 + 1) + b, tanh(a) - b,
            cos(a) + b ** 2, a * b - 1, log1p(a ** 2) - b, atan(a) + sin(b), a / (1 + b ** 2),
            exp(-(a ** 2)) * b, sinh(a) - cosh(b), (a - b) ** 3, a ** 2 * b ** 2 + a,
            expm1(a) * b, sqrt(a ** 2 + b ** 2 + 1)]


def kernel_sweep(k: int, n: int, seed: int = 0) -> Workload:
    """n constraints over consecutive pairs (x_i, x_i+1), i = 0..n-1, split
    into k contiguous blocks, block j using the j-th of the sixteen patterns
    (the kernel-count sweep of Sec. 8.6, Table compile: the size stays fixed
    while the number of distinct patterns varies), plus the objective
    0.5 sum x_i^2."""
    if not 1 <= k <= 16:
        raise ValueError("k must be in 1..16")
    rng = _rng(seed)
    m = Model(f"sweep{k}_{n}")
    x = m.add_var(n + 1, name="x")
    cuts = [n * j // k for j in range(k + 1)]
    for j in range(k):
        d = DataSet(cuts[j + 1] - cuts[j], i=np.arange(cuts[j], cuts[j + 1]))
        m.add_con(_sweep_patterns(x[d.i], x[d.i + 1])[j], d, name=f"k{j}")
    all_pts = DataSet(n + 1, i=np.arange(n + 1))
    m.add_obj(0.5 * x[all_pts.i] ** 2, all_pts, name="reg")
    xv = rng.uniform(-1.0, 1.0, n + 1)
    return Workload(m, xv, rng.standard_normal(m.ncon), 1.0, dict(k=k, n=n))



def two_stage(S: int, n0: int = 8, nz: int = 32, seed: int = 0) -> Workload:
    """Two-stage stochastic model of eq. extensions (one batch instance, S
    scenarios), built with :class:`TwoStageModel`.

    Root: x in R^n0 with the objective 0.5 sum x_i^2 and the rows
    x_i x_{i+1 mod n0} in [-1, 1].  Scenario s (probability 1/S): z_s in
    R^nz, parameters d_s in R^nz (theta), objective (1/S) sum_j (z_js - d_js)^2
    and the rows z_js exp(x_{j mod n0}) - x_{j+1 mod n0}^2 + d_js z_js in
    [-1, 1], so every root variable is touched by about 2 nz S / n0 terms.
    Draw order: d ~ N(0,1); then x ~ U(-1,1), z ~ N(0,1); then y ~ N(0,1).
    """
    from .twostage import TwoStageModel
    rng = _rng(seed)
    m = TwoStageModel(S, f"twostage{S}")
    x = m.add_var(n0, lvar=-5.0, uvar=5.0, name="x")
    z = m.add_var(nz, name="z", each_scenario=True)
    d = m.add_par(rng.standard_normal((nz, S)), name="d", each_scenario=True)
    root = DataSet(n0, i=np.arange(n0), i1=(np.arange(n0) + 1) % n0)
    m.add_obj(0.5 * x[root.i] ** 2, root, name="root_obj")
    m.add_con(x[root.i] * x[root.i1], root, lcon=-1.0, ucon=1.0, name="root_con")
    j = np.tile(np.arange(nz), S)
    s = np.repeat(np.arange(S), nz)
    sc = DataSet(nz * S, k=j + nz * s, xi=j % n0, xn=(j + 1) % n0, scen=s + 1, p=np.full(nz * S, 1.0 / S))
    m.add_obj(sc.p * (z[sc.k] - d[sc.k]) ** 2, sc, name="scen_obj")
    m.add_con(z[sc.k] * exp(x[sc.xi]) - x[sc.xn] ** 2 + d[sc.k] * z[sc.k], sc, lcon=-1.0, ucon=1.0,
              name="scen_con", scenario="scen")
    xv = np.concatenate([rng.uniform(-1.0, 1.0, n0), rng.standard_normal(nz * S)])
    y = rng.standard_normal(m.ncon)
    return Workload(m, xv, y, 1.0, dict(S=S, n0=n0, nz=nz))
