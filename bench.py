"""Benchmark: Jacobian + Hessian nonzeros evaluated per second (FP64).

Workload (default): the ACOPF-shaped synthetic model with 10,000 buses,
13,500 branches and 2,000 generators (seed 1), one instance on one GPU.
One step = every per-iterate callback a solver makes (obj, grad, cons,
jac_coord, hess_coord, jprod, jtprod, hprod) at one iterate, on inputs
already resident in device memory, through one exa_eval call: one
evaluation launch and one reduction launch, outputs bit-identical to the
separate callbacks.  value = (nnzj + nnzh) / step time.

Also reported on the same JSON line:
* step_separate_us -- the same step as seven separate callback calls;
* step_graph_us -- the step captured once into a HIP graph and replayed
  (the paper's protocol times with and without a graph);
* ipm_step_us   -- what an interior-point iteration asks for (obj, grad,
  cons, jac, hess) through one exa_eval call, and its nnz/s;
* callbacks_us  -- each callback alone, timed with the paper's protocol
  (Sec. 8.2: back-to-back calls, one synchronization, best of 3);
* roofline      -- the step's evaluation kernel (exa_k_multi, exa_k_multijh
  with Jacobian + Hessian units, or exa_k_onepass when the tuner picks one
  pass per point for every callback): algorithmic
  bytes per launch / its average duration, measured by HIP events that the
  library records on the launch stream around each launch, against the
  8 TB/s HBM peak; the reduction launch and the combined Jacobian+Hessian
  kernel are reported beside it;
* hbm_copy_gbs  -- a 1 GiB device copy with the library's 16-byte
  non-temporal copy kernel (read + write bytes per second), the practical
  ceiling of a streaming kernel beside the nominal 8 TB/s (torch's copy in
  hbm_copy_torch_gbs);
* rotated       -- the same step cycling over K sets of inputs and outputs
  (>= 512 MB together), so that they come from HBM and not from the 256 MB
  last-level cache (the steady-state step reuses one set, as the paper's
  protocol does);
* cpu_baseline  -- the CPU oracle (numpy, float64) on a bounded sample;
* pde           -- the PDE-control model on a 1000 x 1000 grid
  (HBM-bound): the same step and rooflines;
* batched       -- 256 uneven ACOPF instances (500 to 20,000 buses) in one
  persistent graph-replayed launch vs 256 sequential plain calls;
* adjoint       -- 64 instances of the 10,000-bus model: grad_x L(theta)
  through torch.autograd and its hand-written adjoint, timed against the
  forward and the plain gradient.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Jacobian+Hessian nnz evaluated/sec (FP64, 1e-12 rel); batched vs plain speedup"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the PDE, batched, adjoint, ladder and compile-time legs")
    ap.add_argument("--only", choices=["acopf", "pde", "batch", "adjoint", "ladders", "compile"], default=None,
                    help="run one leg only (used for profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--quick", action="store_true",
                    help="few repetitions per measurement (for runs under a profiler)")
    ap.add_argument("--eval-schedule", default=None,
                    help="block,points_per_lane,fused,units (0 per callback, 1 Jacobian + Hessian units, "
                         "2 one pass): fix the step's exa_eval schedule instead of "
                         "tuning it (to profile the schedule an unprofiled run chose)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB, 5 times (calibrates "
                         "the profiler's HBM byte counters)")
    return ap.parse_args()


# --------------------------------------------------------------- measurement
QUICK = False


def best_of_3(fn, min_s=0.2):
    """The paper's protocol: warm up, N back-to-back calls spanning >= min_s,
    one synchronization, best of three batches.  Returns seconds per call."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    per = max((time.perf_counter() - t0) / 3, 1e-7)
    n = 3 if QUICK else max(3, int(min_s / per))
    best = float("inf")
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / n)
    return best


def kernel_ms(fn, n=200):
    """Average device time of one call: HIP events on the launch stream
    around n back-to-back calls, divided by n.  The queue is first filled with
    a long matrix product so that the host stays ahead of the device and the
    calls run back to back."""
    import torch
    if QUICK:
        n = min(n, 20)
    a = torch.ones(4096, 4096, dtype=torch.float64, device="cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    for _ in range(24):  # ~50 ms of device work, longer than enqueueing n calls
        a = a @ a * 1e-4
    e0.record()
    for _ in range(n):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n, n


def profiled_traffic(summary, model, kernel):
    """HBM bytes per launch of `kernel` measured by rocprofv3 (FETCH_SIZE +
    WRITE_SIZE, calibrated on a plain copy) as committed in profiles/, or
    None when the generated kernels have changed since (their source hash
    differs) or the summary covers another kernel."""
    import hashlib
    from paper_2608_16265_amd import ExaModel
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    src = ExaModel(model, host_only=True).generated_source()
    if hashlib.sha256(src.encode()).hexdigest()[:16] != kv.get("source_sha256_16"):
        return None
    if kv.get("kernel") != kernel:
        return None
    try:
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------- legs
ALL_CBS = ("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod")


def eval_launch_us(em, run, n=500):
    """Average durations (us) of exa_eval's evaluation and reduction launches:
    the library records HIP events on the launch stream around each of its
    launches over n back-to-back calls (the queue is first filled with a long
    matrix product so that the calls run back to back)."""
    import torch
    if QUICK:
        n = min(n, 20)
    a = torch.ones(4096, 4096, dtype=torch.float64, device="cuda:0")
    run()
    torch.cuda.synchronize()
    em.eval_timing(True)
    for _ in range(24):
        a = a @ a * 1e-4
    for _ in range(n):
        run()
    t = em.eval_timing_read()
    em.eval_timing(False)
    return t


def copy_gbs(mib=1024, n=20):
    """Bandwidth (bytes read + written per second) of a 1 GiB device copy,
    with the library's 16-byte non-temporal copy kernel and with torch's:
    the practical ceiling of a streaming kernel on this GPU."""
    import ctypes
    import torch
    from paper_2608_16265_amd import _lib
    a = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    nbytes = a.numel() * 8
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def ours():
        _lib.check(_lib.LIB.exa_device_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                            nbytes, stream))
    out = {}
    for name, fn in (("exa_device_copy", ours), ("torch", lambda: b.copy_(a))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = 2 * nbytes * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
    return out


def _callbacks(em, wl, dev="cuda:0"):
    """Inputs and outputs in device memory for every callback of one model,
    and a zero-argument function per callback.  "eval_all" is every
    per-iterate callback at one point through a single exa_eval call (one
    evaluation launch + one reduction launch), outputs bit-identical to the
    separate callbacks.  Returns (callbacks, (x, y, v, w, jac, hess))."""
    import torch
    X = torch.as_tensor(wl.x, device=dev)
    Y = torch.as_tensor(wl.y, device=dev)
    rng = np.random.default_rng(0)
    V = torch.as_tensor(rng.standard_normal(em.nvar), device=dev)
    W = torch.as_tensor(rng.standard_normal(em.ncon), device=dev)
    e = lambda n: torch.empty(n, dtype=torch.float64, device=dev)  # noqa: E731
    f, g, c, jv, hv = e(1), e(em.nvar), e(em.ncon), e(em.nnzj), e(em.nnzh)
    Jv, Jtw, Hv, Lg = e(em.ncon), e(em.nvar), e(em.nvar), e(em.nvar)
    cbs = {
        "obj": lambda: em.obj(X, f),
        "grad": lambda: em.grad(X, g),
        "cons": lambda: em.cons(X, c),
        "jac_coord": lambda: em.jac_coord(X, jv),
        "hess_coord": lambda: em.hess_coord(X, Y, 1.0, hv),
        "jac_hess_coord": lambda: em.jac_hess_coord(X, Y, 1.0, jv, hv),
        "jprod": lambda: em.jprod(X, V, Jv),
        "jtprod": lambda: em.jtprod(X, W, Jtw),
        "hprod": lambda: em.hprod(X, Y, 1.0, V, Hv),
        "lag_grad": lambda: em.lag_grad(X, Y, 1.0, Lg),
    }
    cbs["eval_all"] = em.bind(X, Y, 1.0, V, W, f=f, g=g, c=c, jac=jv, hess=hv, jv=Jv, jtw=Jtw, hv=Hv)
    # what an interior-point iteration asks for: obj, grad, cons, jac, hess
    cbs["eval_ipm"] = em.bind(X, Y, 1.0, f=f, g=g, c=c, jac=jv, hess=hv)
    return cbs, (X, Y, V, W, jv, hv)


EVAL_SCHEDULE = None


def leg_single(name, wl, steps, warmup):
    import torch
    from paper_2608_16265_amd import ExaModel
    t0 = time.perf_counter()
    em = ExaModel(wl.model, autotune=True)
    build_s = time.perf_counter() - t0
    if EVAL_SCHEDULE:
        b, e_, f_, u_ = (int(v) for v in EVAL_SCHEDULE.split(","))
        em.set_eval_schedule(ALL_CBS, b, e_, bool(f_), u_)
    e = lambda n: torch.empty(n, dtype=torch.float64, device="cuda:0")  # noqa: E731
    cbs, (X, Y, V, W, jv, hv) = _callbacks(em, wl)
    step = cbs["eval_all"]
    # compressed sparse columns from the COO values (the solver-side
    # compression; its structure is analysed once, here)
    for which, coo in (("jac", jv), ("hess", hv)):
        buf = e(int(em.csc_structure(which)[0][-1]))
        cbs[which + "_csc"] = (lambda which=which, coo=coo, buf=buf: em.csc_values(which, coo, buf))
    order = ["obj", "grad", "cons", "jac_hess_coord", "jprod", "jtprod", "hprod"]

    def step_separate():
        for k in order:
            cbs[k]()

    for fn in cbs.values():  # the first call of each tunes its schedule
        fn()
    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / steps
    sep_s = best_of_3(step_separate)
    # HBM-honest variant: K sets of inputs and outputs, >= 512 MB together,
    # used in turn (the model's data and work buffers stay as they are)
    per_set = 8 * (2 * em.nvar + 2 * em.ncon + 1 + em.nvar + em.ncon + em.nnzj + em.nnzh + em.ncon + 2 * em.nvar)
    K = max(2, -(-(512 << 20) // per_set))
    sets = []
    for _ in range(K):
        Xk, Yk = X.clone(), Y.clone()
        Vk, Wk = V.clone(), W.clone()
        sets.append(em.bind(Xk, Yk, 1.0, Vk, Wk, f=e(1), g=e(em.nvar), c=e(em.ncon), jac=e(em.nnzj),
                            hess=e(em.nnzh), jv=e(em.ncon), jtw=e(em.nvar), hv=e(em.nvar)))
    for fn in sets:
        fn()
    torch.cuda.synchronize()
    nrot = max(K, steps // K * K)
    t0 = time.perf_counter()
    for i in range(nrot):
        sets[i % K]()
    torch.cuda.synchronize()
    rot_s = (time.perf_counter() - t0) / nrot
    del sets
    # the paper's protocol times with and without a graph: the step captured
    # once into a HIP graph (torch.cuda.CUDAGraph) and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    graph_s = best_of_3(g.replay)
    per_cb = {k: best_of_3(fn) * 1e6 for k, fn in cbs.items()}
    tm = eval_launch_us(em, step)
    eb = em.eval_bytes(ALL_CBS)
    k_mean, k_n = kernel_ms(cbs["jac_hess_coord"])
    rd, wr = em.kernel_bytes("jac_hess")
    sched = {k: em.schedule(k) for k in ("jac", "hess", "jac_hess")}
    sched["eval_all"] = em.eval_schedule(ALL_CBS)
    # the tuner picks per-callback tiles (exa_k_multi, or exa_k_multijh with
    # Jacobian + Hessian units) or one pass per point
    # for every callback (exa_k_onepass)
    sa = sched["eval_all"]
    eval_kernel = "exa_k_onepass" if sa["one_pass"] else "exa_k_multijh" if sa["jac_hess"] else "exa_k_multi"
    nnz = em.nnzj + em.nnzh
    ev_bytes = eb["eval_read"] + eb["eval_write"]
    red_bytes = eb["reduce_read"] + eb["reduce_write"]
    res = dict(
        name=name, nvar=em.nvar, ncon=em.ncon, nnzj=em.nnzj, nnzh=em.nnzh,
        build_s=round(build_s, 3), step_s=step_s, nnz_per_s=nnz / step_s,
        step_separate_us=round(sep_s * 1e6, 2), step_graph_us=round(graph_s * 1e6, 2),
        rotated=dict(sets=K, mb=round(K * per_set / 1e6, 1), step_us=round(rot_s * 1e6, 2),
                     nnz_per_s=(em.nnzj + em.nnzh) / rot_s),
        jac_hess_nnz_per_s=nnz / (per_cb["jac_hess_coord"] * 1e-6),
        ipm_step_us=round(per_cb["eval_ipm"], 2), ipm_nnz_per_s=nnz / (per_cb["eval_ipm"] * 1e-6),
        jac_plus_hess_nnz_per_s=nnz / ((per_cb["jac_coord"] + per_cb["hess_coord"]) * 1e-6),
        callbacks_us={k: round(v, 2) for k, v in per_cb.items()},
        eval_kernel=eval_kernel, eval_us=round(tm["eval_us"], 3), eval_calls_timed=tm["calls"],
        reduce_us=round(tm["reduce_us"], 3),
        eval_bytes=ev_bytes, eval_read_bytes=eb["eval_read"], eval_write_bytes=eb["eval_write"],
        reduce_bytes=red_bytes,
        eval_gbs=ev_bytes / (tm["eval_us"] * 1e-6) / 1e9,
        reduce_gbs=red_bytes / (tm["reduce_us"] * 1e-6) / 1e9 if tm["reduce_us"] > 0 else None,
        jh_kernel_us=round(k_mean * 1e3, 3), kernel_launches_timed=k_n,
        jh_bytes=rd + wr, jh_gbs=(rd + wr) / (k_mean * 1e-3) / 1e9,
        schedule=sched,
    )
    em.close()
    return res


def leg_batch(count=256, first_seed=1000):
    import torch
    from exa_modeling.generators import acopf_batch
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    t0 = time.perf_counter()
    wls = acopf_batch(count, first_seed)
    ems = []
    for i, w in enumerate(wls):
        ems.append(ExaModel(w.model))
        if (i + 1) % 64 == 0:
            log(f"  batch: {i + 1}/{count} models built")
    build_s = time.perf_counter() - t0
    b = ExaBatch(ems, autotune=True)
    X = b.concat_x([w.x for w in wls])
    Y = b.concat_y([w.y for w in wls])
    J = torch.empty(b.total("jac"), dtype=torch.float64, device="cuda:0")
    H = torch.empty(b.total("hess"), dtype=torch.float64, device="cuda:0")
    b.eval(X, Y, 1.0, J, H)  # tunes the schedule, records the graph
    torch.cuda.synchronize()
    t_batch = best_of_3(lambda: b.eval(X, Y, 1.0, J, H))
    xs = [torch.as_tensor(w.x, device="cuda:0") for w in wls]
    ys = [torch.as_tensor(w.y, device="cuda:0") for w in wls]
    js = [torch.empty(e.nnzj, dtype=torch.float64, device="cuda:0") for e in ems]
    hs = [torch.empty(e.nnzh, dtype=torch.float64, device="cuda:0") for e in ems]

    def plain():
        for e, x, y, j, h in zip(ems, xs, ys, js, hs):
            e.jac_coord(x, j)
            e.hess_coord(x, y, 1.0, h)

    t_plain = best_of_3(plain, min_s=0.3)
    nnz = b.total("jac") + b.total("hess")
    # identical results, instance by instance
    torch.cuda.synchronize()
    same = True
    off = b.offsets()
    for i in range(0, count, 17):
        same &= bool(torch.equal(J[off[i, 2]:off[i + 1, 2]], js[i]))
        same &= bool(torch.equal(H[off[i, 3]:off[i + 1, 3]], hs[i]))
    sched = b.schedule()
    k_mean, _ = kernel_ms(lambda: b.eval(X, Y, 1.0, J, H), n=50)
    rd, wr = b.kernel_bytes()
    res = dict(instances=count, buses=int(sum(w.meta["nb"] for w in wls)), nnz=int(nnz),
               build_s=round(build_s, 2), batched_us=round(t_batch * 1e6, 1),
               plain_us=round(t_plain * 1e6, 1), speedup=t_plain / t_batch,
               batched_nnz_per_s=nnz / t_batch, plain_nnz_per_s=nnz / t_plain,
               bitwise_equal_sampled=same, schedule=sched,
               kernel_us=round(k_mean * 1e3, 1), read_bytes=rd, write_bytes=wr,
               roofline={"kernel": "exa_k_jh", "bound": "hbm",
                         "achieved": (rd + wr) / (k_mean * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": (rd + wr) / (k_mean * 1e-3) / 1e9 / HBM_PEAK_GBS})
    b.close()
    for e in ems:
        e.close()
    return res


def leg_adjoint(count=64, first_seed=2000):
    """64 instances of the 10,000-bus model: the Lagrangian gradient as a
    function of theta (forward) and its hand-written adjoint (backward),
    through torch.autograd, vs the plain gradient callback."""
    import torch
    from exa_modeling.generators import acopf
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.adjoint import lagrangian_gradient
    t0 = time.perf_counter()
    wls, ems = [], []
    for i in range(count):
        wls.append(acopf(10000, first_seed + i))
        ems.append(ExaModel(wls[-1].model))
        if (i + 1) % 16 == 0:
            log(f"  adjoint: {i + 1}/{count} models built")
    build_s = time.perf_counter() - t0
    dev = "cuda:0"
    xs = [torch.as_tensor(w.x, device=dev) for w in wls]
    ys = [torch.as_tensor(w.y, device=dev) for w in wls]
    ths = [torch.as_tensor(w.model.theta, device=dev).requires_grad_(True) for w in wls]
    ws = [torch.as_tensor(np.random.default_rng(first_seed + i).standard_normal(e.nvar), device=dev)
          for i, e in enumerate(ems)]
    gs = [torch.empty(e.nvar, dtype=torch.float64, device=dev) for e in ems]

    def forward():
        return [lagrangian_gradient(th, e, x, y, 1.0) for th, e, x, y in zip(ths, ems, xs, ys)]

    def fwd_bwd():
        outs = forward()
        torch.autograd.backward(outs, ws)

    def backward_only():
        for th, e, x, y, w in zip(ths, ems, xs, ys, ws):
            e.adjoint_theta(x, y, 1.0, w)

    def grad_only():
        for e, x, g in zip(ems, xs, gs):
            e.grad(x, g)

    t_fwd = best_of_3(lambda: forward(), min_s=0.2)
    t_fb = best_of_3(fwd_bwd, min_s=0.2)
    t_bwd = best_of_3(backward_only, min_s=0.2)
    t_grad = best_of_3(grad_only, min_s=0.2)
    return dict(instances=count, buses_each=10000, ntheta_each=ems[0].ntheta,
                build_s=round(build_s, 2), forward_us=round(t_fwd * 1e6, 1),
                forward_backward_us=round(t_fb * 1e6, 1), adjoint_kernel_path_us=round(t_bwd * 1e6, 1),
                grad_us=round(t_grad * 1e6, 1), backward_over_forward=t_bwd / t_fwd,
                backward_over_grad=t_bwd / t_grad)


LADDER_CBS = ("obj", "grad", "cons", "jac_coord", "hess_coord", "jac_hess_coord", "jprod", "jtprod", "hprod",
              "eval_all")


def leg_ladders():
    """Single instances as they grow (the per-instance scaling study of
    Sec. 8): every callback's time, by the paper's protocol, on the extended
    Rosenbrock objective of eq. rosenbrock at N = 20, 2,000 and 200,000, the
    ACOPF-shaped model at 118, 1,354 and 78,484 buses, the Goddard rocket
    of eq. rocket at T = 200, 20,000 and 2,000,000 steps, and a two-stage
    stochastic model (8 root variables, 32 per scenario) at 64, 4,096 and
    65,536 scenarios.  Each model's every callback is one evaluation launch
    plus at most one reduction launch (one more where a variable is shared
    by more than 1,024 terms), whatever its number of patterns."""
    import torch
    from exa_modeling.generators import acopf, goddard, rosenbrock, two_stage
    from paper_2608_16265_amd import ExaModel
    out = {}
    for fam, sizes, make in (("rosenbrock", (20, 2000, 200000), lambda N: rosenbrock(N, 0)),
                             ("acopf", (118, 1354, 78484), lambda nb: acopf(nb, 5)),
                             ("goddard", (200, 20000, 2000000), lambda T: goddard(T, 0)),
                             ("two_stage", (64, 4096, 65536), lambda S: two_stage(S, 8, 32, 0))):
        rows = []
        for size in sizes:
            wl = make(size)
            em = ExaModel(wl.model, autotune=True)
            cbs, _ = _callbacks(em, wl)
            for fn in cbs.values():  # the first call of each tunes its schedule
                fn()
            torch.cuda.synchronize()
            t = {k: round(best_of_3(cbs[k], min_s=0.1) * 1e6, 2) for k in LADDER_CBS}
            nnz = em.nnzj + em.nnzh
            rows.append(dict(size=size, nvar=em.nvar, ncon=em.ncon, nnzj=em.nnzj, nnzh=em.nnzh,
                             patterns=len(wl.model.patterns), callbacks_us=t,
                             jac_plus_hess_nnz_per_s=nnz / ((t["jac_coord"] + t["hess_coord"]) * 1e-6)))
            log(f"  ladder {fam} {size}: " + json.dumps(t))
            em.close()
            del cbs
        out[fam] = rows
    return out


def _compile_point(k, n):
    """Build cost of the kernel-sweep model with k distinct constraint
    patterns over n pairs: host analysis and code generation alone
    (host_ms), creation with run-time compilation and module load (cold:
    no live model shares its patterns), the first exa_eval of every callback
    (first_eval_ms), and creation while a model with the same patterns is
    alive (cached: the compiled module is shared, nothing is compiled)."""
    import torch
    from exa_modeling.generators import kernel_sweep
    from paper_2608_16265_amd import ExaModel
    wl = kernel_sweep(k, n, 0)
    t0 = time.perf_counter()
    h = ExaModel(wl.model, host_only=True)
    host_s = time.perf_counter() - t0
    src_kb = len(h.generated_source()) / 1024
    h.close()
    t0 = time.perf_counter()
    em = ExaModel(wl.model)
    create_s = time.perf_counter() - t0
    cbs, _ = _callbacks(em, wl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cbs["eval_all"]()
    torch.cuda.synchronize()
    first_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    em2 = ExaModel(wl.model)
    cached_s = time.perf_counter() - t0
    res = dict(kernels=k, n=n, patterns=len(wl.model.patterns), nnzj=em.nnzj, nnzh=em.nnzh,
               source_kb=round(src_kb, 1), host_ms=round(host_s * 1e3, 1), create_ms=round(create_s * 1e3, 1),
               first_eval_ms=round(first_s * 1e3, 2), create_cached_ms=round(cached_s * 1e3, 1))
    em2.close()
    em.close()
    log("  compile " + json.dumps(res))
    return res


def leg_compile():
    """Model build time (the compilation study of Sec. 8, Table compile):
    the number of distinct constraint patterns swept over 1, 2, 4, 8 and 16
    at 100,000 constraints, and the size swept over 1,000 to 1,000,000
    constraints at four patterns."""
    return dict(kernels=[_compile_point(k, 100000) for k in (1, 2, 4, 8, 16)],
                size=[_compile_point(4, n) for n in (1000, 10000, 100000, 1000000)])


def cpu_baseline(wl, seconds):
    """The CPU oracle as it stands, timed on a bounded sample of the same
    workload: repeated full jac_coord + hess_coord of the 10k-bus model."""
    from oracle import OracleModel
    o = OracleModel(wl.model)
    o.jac_coord(wl.x)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.jac_coord(wl.x)
        o.hess_coord(wl.x, wl.y, 1.0)
        n += 1
        if time.perf_counter() - t0 >= seconds:
            break
    per = (time.perf_counter() - t0) / n
    nnz = o.nnzj + o.nnzh
    return dict(value=nnz / per, unit="nnz/s", cores=1, kind="oracle",
                sample=f"{n} x (jac_coord + hess_coord) of the full 10,000-bus model, "
                       f"{per:.3f} s each, numpy float64 single thread")


def copy_only(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8}))


def main():
    global QUICK, EVAL_SCHEDULE
    args = parse()
    QUICK = args.quick
    EVAL_SCHEDULE = args.eval_schedule
    if args.copy_mib:
        copy_only(args.copy_mib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(instances of a batch would be sharded across GPUs with no exchange; not implemented).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from exa_modeling.generators import acopf, pde

    out = {"metric": METRIC, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if args.only in (None, "acopf"):
        log("leg: acopf 10k")
        wl = acopf(10000, 1)
        r = leg_single("acopf10k", wl, args.steps, args.warmup)
        log(json.dumps(r))
        out.update(value=r["nnz_per_s"], ms_per_step=r["step_s"] * 1e3)
        out["config"] = {"workload": "acopf-10000-bus (13,500 branches, 2,000 generators, seed 1)",
                         "step": "exa_eval of obj, grad, cons, jac, hess, jprod, jtprod, hprod at one iterate",
                         "nvar": r["nvar"], "ncon": r["ncon"], "nnzj": r["nnzj"],
                         "nnzh": r["nnzh"], "schedule": r["schedule"]}
        out["step_separate_us"] = r["step_separate_us"]
        out["step_graph_us"] = r["step_graph_us"]
        out["rotated"] = r["rotated"]
        out["callbacks_us"] = r["callbacks_us"]
        out["jac_hess_nnz_per_s"] = r["jac_hess_nnz_per_s"]
        out["ipm_step_us"] = r["ipm_step_us"]
        out["ipm_nnz_per_s"] = r["ipm_nnz_per_s"]
        out["jac_plus_hess_nnz_per_s"] = r["jac_plus_hess_nnz_per_s"]
        from exa_modeling.generators import acopf as _acopf
        traffic = profiled_traffic("acopf10k_eval_all.md", _acopf(30, 0).model, r["eval_kernel"])
        out["roofline"] = {"kernel": r["eval_kernel"], "bound": "hbm", "achieved": r["eval_gbs"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": r["eval_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                           "bytes_per_launch": r["eval_bytes"], "read_bytes": r["eval_read_bytes"],
                           "write_bytes": r["eval_write_bytes"], "launch_us": r["eval_us"],
                           "launches_timed": r["eval_calls_timed"]}
        out["roofline_reduce"] = {"kernel": "k_reduce", "achieved": r["reduce_gbs"],
                                  "bytes_per_launch": r["reduce_bytes"], "launch_us": r["reduce_us"]}
        out["roofline_jac_hess_coord"] = {"kernel": "exa_k_jh", "achieved": r["jh_gbs"],
                                          "frac": r["jh_gbs"] / HBM_PEAK_GBS,
                                          "bytes_per_launch": r["jh_bytes"], "launch_us": r["jh_kernel_us"]}
        cg = copy_gbs()
        out["hbm_copy_gbs"] = cg["exa_device_copy"]
        out["hbm_copy_torch_gbs"] = cg["torch"]
        if not args.no_cpu_baseline:
            log("leg: cpu baseline")
            out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    if not args.no_extras and args.only in (None, "pde"):
        log("leg: pde 1000")
        wl = pde(1000, 3)
        r = leg_single("pde1000", wl, max(20, args.steps // 20), 5)
        log(json.dumps(r))
        out["pde"] = {"workload": "pde-control 1000x1000 grid (2e6 variables, seed 3)",
                      "nnzj": r["nnzj"], "nnzh": r["nnzh"], "step_us": round(r["step_s"] * 1e6, 2),
                      "nnz_per_s": r["nnz_per_s"], "step_separate_us": r["step_separate_us"],
                      "step_graph_us": r["step_graph_us"],
                      "rotated": r["rotated"],
                      "jac_hess_nnz_per_s": r["jac_hess_nnz_per_s"],
                      "ipm_step_us": r["ipm_step_us"], "ipm_nnz_per_s": r["ipm_nnz_per_s"],
                      "callbacks_us": r["callbacks_us"],
                      "roofline_eval": {"kernel": r["eval_kernel"], "achieved": r["eval_gbs"],
                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": r["eval_gbs"] / HBM_PEAK_GBS,
                                        "bytes_per_launch": r["eval_bytes"], "launch_us": r["eval_us"]},
                      "roofline_reduce": {"kernel": "k_reduce", "achieved": r["reduce_gbs"],
                                          "bytes_per_launch": r["reduce_bytes"], "launch_us": r["reduce_us"]},
                      "roofline_jh": {"kernel": "exa_k_jh", "achieved": r["jh_gbs"],
                                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": r["jh_gbs"] / HBM_PEAK_GBS,
                                      "bytes_per_launch": r["jh_bytes"],
                                      "launch_us": r["jh_kernel_us"]}}
        if args.only == "pde":
            out.update(value=r["nnz_per_s"], ms_per_step=r["step_s"] * 1e3)
    if not args.no_extras and args.only in (None, "batch"):
        log("leg: batched 256")
        r = leg_batch()
        log(json.dumps(r))
        out["batched"] = r
        if args.only == "batch":
            out.update(value=r["batched_nnz_per_s"], ms_per_step=r["batched_us"] * 1e-3)
    if not args.no_extras and args.only in (None, "adjoint"):
        log("leg: adjoint 64 x 10k")
        r = leg_adjoint()
        log(json.dumps(r))
        out["adjoint"] = r
    if not args.no_extras and args.only in (None, "ladders"):
        log("leg: per-instance ladders")
        out["ladders"] = leg_ladders()
    if not args.no_extras and args.only in (None, "compile"):
        log("leg: build time vs patterns and size")
        out["compile"] = leg_compile()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
