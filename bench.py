"""Benchmark: Jacobian + Hessian nonzeros evaluated per second (FP64).

Workload (default headline): 256 ACOPF-shaped synthetic instances of uneven
size (buses log-uniform in 500-20,000, loads perturbed by U(0.9, 1.1),
seeds 1000-1255), the batched configuration, on one GPU.  One step = every
per-iterate callback a solver makes (obj, grad, cons, jac_coord,
hess_coord, jprod, jtprod, hprod) for every instance at one iterate, on
inputs already resident in device memory, through one exa_batch_eval call
replayed from a HIP graph: one evaluation launch over every instance's
tiles and one launch of every instance's reductions, each instance's
outputs bit-identical to its own callbacks.
value = sum over instances of (nnzj + nnzh) / step time.

Also reported on the same JSON line:
* batched       -- the same batch against the plain per-instance path: 256
  exa_eval calls of every callback, 256 exa_jac_hess_coord calls, 256
  exa_jac_coord + exa_hess_coord pairs, and the batched Jacobian + Hessian
  alone; speedups, and a bitwise check of every instance's every output;
* roofline      -- the step's evaluation launch: algorithmic bytes per
  launch / its average duration, from HIP events that the library records
  on the launch stream around each launch, against the 8 TB/s HBM peak
  (traffic: rocprofv3 FETCH_SIZE + WRITE_SIZE of the committed profile);
  the reduction launch beside it;
* cpu_baseline  -- the CPU oracle (numpy, float64) on a bounded sample of
  the same workload: every callback of whole instances, one process and
  one process per core (before the GPU is touched);
* acopf10k, pde -- one 10,000-bus ACOPF instance and the PDE-control model
  on a 1000 x 1000 grid: the same step through exa_eval, graph replay,
  separate callbacks, rotated buffers, rooflines;
* adjoint       -- 64 instances of the 10,000-bus model: grad_x L(theta)
  of all of them as one torch.autograd.Function over the batch and its
  hand-written adjoint, timed against the forward and the plain gradient;
* ladders, compile -- per-instance scaling and build time.
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
    ap.add_argument("--only", choices=["batch", "acopf", "pde", "adjoint", "ladders", "compile"], default=None,
                    help="run one leg only (used for profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--quick", action="store_true",
                    help="few repetitions per measurement (for runs under a profiler)")
    ap.add_argument("--eval-schedule", default=None,
                    help="block,points_per_lane,fused,units[,unstaged] (units 0 per callback, 1 Jacobian + "
                         "Hessian units, 2 one pass; unstaged 1: each lane's own stores): fix the step's exa_eval "
                         "schedule instead of tuning it (to profile the schedule an unprofiled run chose)")
    ap.add_argument("--batch-schedule", default=None,
                    help="block,points_per_lane,fused,units[,unstaged] (units per_callback, jac_hess, one_pass "
                         "or separate; unstaged 1: each lane's own stores): fix the headline batch step's "
                         "schedule instead of tuning it (to profile the schedule an unprofiled run chose)")
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
    WRITE_SIZE, calibrated on a plain copy) as committed in profiles/, with
    the schedule the counted launches ran; (None, None) when the generated
    kernels have changed since (their source hash differs) or the summary
    covers another kernel."""
    import hashlib
    from paper_2608_16265_amd import ExaModel
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None, None
    kv = {}
    for line in open(path):
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    src = ExaModel(model, host_only=True).generated_source()
    if hashlib.sha256(src.encode()).hexdigest()[:16] != kv.get("source_sha256_16"):
        return None, None
    if kv.get("kernel") != kernel:
        return None, None
    try:
        return int(kv["traffic_bytes_per_launch"]), kv.get("schedule")
    except (KeyError, ValueError):
        return None, None


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
BATCH_SCHEDULE = None


def leg_single(name, wl, steps, warmup):
    import torch
    from paper_2608_16265_amd import ExaModel
    t0 = time.perf_counter()
    em = ExaModel(wl.model, autotune=True)
    build_s = time.perf_counter() - t0
    if EVAL_SCHEDULE:
        v = [int(t) for t in EVAL_SCHEDULE.split(",")]
        em.set_eval_schedule(ALL_CBS, v[0], v[1], bool(v[2]), v[3], unstaged=len(v) > 4 and bool(v[4]))
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


ALL8 = dict(f="B", g="x", c="y", jac="jac", hess="hess", jv="y", jtw="x", hv="x")
BATCH_CBS = ("obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod")


def batch_launch_us(b, run, n=50):
    """Average durations (us) of the batched evaluation and reduction
    launches: with timing on, the library launches directly and records HIP
    events on the launch stream around each launch; the queue is first
    filled with a long matrix product so that the calls run back to back."""
    import torch
    if QUICK:
        n = min(n, 5)
    a = torch.ones(4096, 4096, dtype=torch.float64, device="cuda:0")
    b.timing(True)
    run()
    torch.cuda.synchronize()
    b.timing_read()
    for _ in range(24):
        a = a @ a * 1e-4
    for _ in range(n):
        run()
    t = b.timing_read()
    b.timing(False)
    return t


def leg_batch(steps, warmup, count=256, first_seed=1000):
    """The headline: all callbacks of 256 uneven instances per step."""
    import torch
    from exa_modeling.generators import acopf_batch
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.batch import ExaBatch
    t0 = time.perf_counter()
    wls = acopf_batch(count, first_seed)
    ems = []
    for i, w in enumerate(wls):
        # tuned per instance: the plain baseline is each instance's fastest
        # exa_eval (the batch tunes its own schedule)
        ems.append(ExaModel(w.model, autotune=True))
        if (i + 1) % 64 == 0:
            log(f"  batch: {i + 1}/{count} models built")
    build_s = time.perf_counter() - t0
    b = ExaBatch(ems, autotune=True)
    if BATCH_SCHEDULE:
        v = BATCH_SCHEDULE.split(",")
        b.set_schedule(BATCH_CBS, int(v[0]), int(v[1]), bool(int(v[2])), v[3],
                       unstaged=len(v) > 4 and bool(int(v[4])))
    dev = "cuda:0"
    rng = np.random.default_rng(0)
    X = b.concat([w.x for w in wls])
    Y = b.concat([w.y for w in wls])
    V = torch.as_tensor(rng.standard_normal(b.total("x")), device=dev)
    W = torch.as_tensor(rng.standard_normal(b.total("y")), device=dev)
    outs = {k: b.empty(kind) for k, kind in ALL8.items()}
    step = b.bind(X, Y, 1.0, V, W, **outs)
    t0 = time.perf_counter()
    step()  # tunes the schedule, records the graph
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / steps
    log(f"  batch step {step_s * 1e6:.1f} us")
    tm = batch_launch_us(b, step)
    eb = b.kernel_bytes(BATCH_CBS)
    sched = b.schedule(BATCH_CBS)
    eval_kernel = ("exa_k_onepass" if sched["units"] == "one_pass" else
                   "exa_k_multijh" if sched["units"] == "jac_hess" else "exa_k_multi")
    # the batched Jacobian + Hessian alone (the metric's own pair)
    J, H = b.empty("jac"), b.empty("hess")
    jh = b.bind(X, Y, 1.0, jac=J, hess=H)
    jh()
    torch.cuda.synchronize()
    t_jh = best_of_3(jh)
    jh_sched = b.schedule(("jac", "hess"))
    jh_bytes = b.kernel_bytes(("jac", "hess"))
    jh_tm = batch_launch_us(b, jh)
    # the plain per-instance path on the same data
    off = b.offsets()
    xs = [X[b.slice("x", i)].clone() for i in range(count)]
    ys = [Y[b.slice("y", i)].clone() for i in range(count)]
    vs = [V[b.slice("x", i)].clone() for i in range(count)]
    ws = [W[b.slice("y", i)].clone() for i in range(count)]
    e = lambda n: torch.empty(n, dtype=torch.float64, device=dev)  # noqa: E731
    plain_outs = [dict(f=e(1), g=e(m.nvar), c=e(m.ncon), jac=e(m.nnzj), hess=e(m.nnzh), jv=e(m.ncon),
                       jtw=e(m.nvar), hv=e(m.nvar)) for m in ems]
    binds = [m.bind(x, y, 1.0, v, w, **o) for m, x, y, v, w, o in zip(ems, xs, ys, vs, ws, plain_outs)]
    for f in binds:
        f()
    torch.cuda.synchronize()

    def plain_all():
        for f in binds:
            f()

    def plain_jh():
        for m, x, y, o in zip(ems, xs, ys, plain_outs):
            m.jac_hess_coord(x, y, 1.0, o["jac"], o["hess"])

    def plain_two():
        for m, x, y, o in zip(ems, xs, ys, plain_outs):
            m.jac_coord(x, o["jac"])
            m.hess_coord(x, y, 1.0, o["hess"])

    t_plain_all = best_of_3(plain_all, min_s=0.3)
    t_plain_jh = best_of_3(plain_jh, min_s=0.3)
    t_plain_two = best_of_3(plain_two, min_s=0.3)
    # every instance's every output, bit for bit
    for f in binds:
        f()
    step()
    torch.cuda.synchronize()
    same = True
    for i in range(count):
        for k, kind in ALL8.items():
            sl = slice(i, i + 1) if kind == "B" else b.slice(kind, i)
            same &= bool(torch.equal(outs[k][sl], plain_outs[i][k]))
    same_jh = all(bool(torch.equal(J[b.slice("jac", i)], plain_outs[i]["jac"])) and
                  bool(torch.equal(H[b.slice("hess", i)], plain_outs[i]["hess"])) for i in range(count))
    nnz = b.total("jac") + b.total("hess")
    ev_bytes = eb["eval_read"] + eb["eval_write"]
    red_bytes = eb["reduce_read"] + eb["reduce_write"]
    res = dict(
        instances=count, buses=int(sum(w.meta["nb"] for w in wls)),
        nvar=b.total("x"), ncon=b.total("y"), nnzj=b.total("jac"), nnzh=b.total("hess"), nnz=int(nnz),
        build_s=round(build_s, 2), first_call_s=round(tune_s, 2),
        step_s=step_s, nnz_per_s=nnz / step_s, schedule=sched, eval_kernel=eval_kernel,
        eval_us=round(tm["eval_us"], 2), reduce_us=round(tm["reduce_us"], 2), launches_timed=tm["calls"],
        eval_read_bytes=eb["eval_read"], eval_write_bytes=eb["eval_write"], eval_bytes=ev_bytes,
        reduce_bytes=red_bytes, eval_gbs=ev_bytes / (tm["eval_us"] * 1e-6) / 1e9,
        reduce_gbs=red_bytes / (tm["reduce_us"] * 1e-6) / 1e9 if tm["reduce_us"] > 0 else None,
        plain_eval_all_us=round(t_plain_all * 1e6, 1), speedup_vs_plain_eval_all=t_plain_all / step_s,
        batched_jac_hess_us=round(t_jh * 1e6, 1), batched_jac_hess_nnz_per_s=nnz / t_jh,
        jac_hess_schedule=jh_sched, jac_hess_eval_us=round(jh_tm["eval_us"], 2),
        jac_hess_bytes=jh_bytes["eval_read"] + jh_bytes["eval_write"],
        jac_hess_gbs=(jh_bytes["eval_read"] + jh_bytes["eval_write"]) / (jh_tm["eval_us"] * 1e-6) / 1e9,
        plain_jac_hess_coord_us=round(t_plain_jh * 1e6, 1),
        plain_jac_then_hess_us=round(t_plain_two * 1e6, 1),
        speedup_jac_hess_vs_plain_jac_hess_coord=t_plain_jh / t_jh,
        speedup_jac_hess_vs_plain_jac_then_hess=t_plain_two / t_jh,
        bitwise_equal_all_instances=bool(same), bitwise_equal_jac_hess=bool(same_jh))
    del off
    b.close()
    for m in ems:
        m.close()
    return res


def leg_adjoint(count=64, first_seed=2000):
    """64 instances of the 10,000-bus model: the Lagrangian gradients as one
    function of the concatenated parameters (forward: one batched call of
    EXA_EV_LAG), its hand-written adjoint (backward: one batched call of
    EXA_EV_ADJ), through torch.autograd, vs the plain gradient."""
    import torch
    from exa_modeling.generators import acopf
    from paper_2608_16265_amd import ExaModel
    from paper_2608_16265_amd.adjoint import batch_lagrangian_gradient, lagrangian_gradient
    from paper_2608_16265_amd.batch import ExaBatch
    t0 = time.perf_counter()
    wls, ems = [], []
    for i in range(count):
        wls.append(acopf(10000, first_seed + i))
        ems.append(ExaModel(wls[-1].model))
        if (i + 1) % 16 == 0:
            log(f"  adjoint: {i + 1}/{count} models built")
    build_s = time.perf_counter() - t0
    dev = "cuda:0"
    b = ExaBatch(ems, autotune=True)
    X = b.concat([w.x for w in wls])
    Y = b.concat([w.y for w in wls])
    TH = b.concat([w.model.theta for w in wls])
    theta = TH.clone().requires_grad_(True)
    Wc = torch.as_tensor(np.concatenate([np.random.default_rng(first_seed + i).standard_normal(e.nvar)
                                         for i, e in enumerate(ems)]), device=dev)
    G = b.empty("x")
    TB = b.empty("theta")
    grad_only = b.bind(X, Y, 1.0, g=G)
    adj_only = b.bind(X, Y, 1.0, wx=Wc, theta_bar=TB)

    def forward():
        return batch_lagrangian_gradient(theta, b, X, Y, 1.0)

    def fwd_bwd():
        out = forward()
        torch.autograd.backward(out, Wc)

    for fn in (forward, fwd_bwd, grad_only, adj_only):  # first calls tune and record
        fn()
    torch.cuda.synchronize()
    t_fwd = best_of_3(forward, min_s=0.2)
    t_fb = best_of_3(fwd_bwd, min_s=0.2)
    t_bwd = best_of_3(adj_only, min_s=0.2)
    t_grad = best_of_3(grad_only, min_s=0.2)
    # the per-instance path it replaces: 64 autograd nodes over 64 models
    xs = [X[b.slice("x", i)].clone() for i in range(count)]
    ys = [Y[b.slice("y", i)].clone() for i in range(count)]
    ths = [TH[b.slice("theta", i)].clone().requires_grad_(True) for i in range(count)]
    wss = [Wc[b.slice("x", i)].clone() for i in range(count)]

    def per_instance_fb():
        outs = [lagrangian_gradient(th, e, x, y, 1.0) for th, e, x, y in zip(ths, ems, xs, ys)]
        torch.autograd.backward(outs, wss)

    t_pi = best_of_3(per_instance_fb, min_s=0.2)
    b.close()
    return dict(instances=count, buses_each=10000, ntheta_each=ems[0].ntheta,
                build_s=round(build_s, 2), forward_us=round(t_fwd * 1e6, 1),
                forward_backward_us=round(t_fb * 1e6, 1), adjoint_kernel_path_us=round(t_bwd * 1e6, 1),
                grad_us=round(t_grad * 1e6, 1), backward_over_forward=t_bwd / t_fwd,
                backward_over_grad=t_bwd / t_grad,
                autograd_overhead_us=round((t_fb - t_fwd - t_bwd) * 1e6, 1),
                per_instance_forward_backward_us=round(t_pi * 1e6, 1))


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


_CACHE_CHILD = """
import json, sys, time
sys.path.insert(0, {root!r})
from exa_modeling.generators import kernel_sweep
from paper_2608_16265_amd import ExaModel
w = kernel_sweep({k}, 100000, 0)
t0 = time.perf_counter()
em = ExaModel(w.model, cache_dir={d!r})
print(json.dumps(dict(create_ms=(time.perf_counter() - t0) * 1e3, **em.build_info())))
"""


def _cache_processes(k):
    """Create of the k-pattern sweep model in a fresh process with an empty
    on-disk code-object cache, then in a second fresh process that finds it
    there."""
    import subprocess
    import tempfile
    out = []
    with tempfile.TemporaryDirectory() as d:
        for _ in range(2):
            r = subprocess.run([sys.executable, "-c", _CACHE_CHILD.format(root=ROOT, k=k, d=d)],
                               capture_output=True, text=True, timeout=300)
            if r.returncode != 0:
                return {"error": r.stderr[-500:]}
            out.append(json.loads(r.stdout.strip().splitlines()[-1]))
    return dict(kernels=k, first_process=out[0], second_process=out[1])


def leg_compile():
    """Model build time (the compilation study of Sec. 8, Table compile):
    the number of distinct constraint patterns swept over 1, 2, 4, 8 and 16
    at 100,000 constraints, the size swept over 1,000 to 1,000,000
    constraints at four patterns, and a second process reading the
    16-pattern code object from the on-disk cache."""
    return dict(kernels=[_compile_point(k, 100000) for k in (1, 2, 4, 8, 16)],
                size=[_compile_point(4, n) for n in (1000, 10000, 100000, 1000000)],
                disk_cache=_cache_processes(16))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_instances(worker, workers, seconds, first_seed=1000, count=256):
    """Every callback of whole instances of the batch workload through the
    oracle as it stands (instances worker, worker + workers, ...), until
    `seconds` of timed work; setup (drawing the instance and the oracle's
    structure analysis) is not timed.  Returns (nnz, timed seconds,
    instances)."""
    from exa_modeling.generators import acopf_batch_instance
    from oracle import OracleModel
    nnz, busy, n = 0, 0.0, 0
    i = worker
    while busy < seconds and i < count:
        w = acopf_batch_instance(first_seed + i)
        o = OracleModel(w.model)
        rng = np.random.default_rng(i)
        v, wv = rng.standard_normal(o.nvar), rng.standard_normal(o.ncon)
        t0 = time.perf_counter()
        o.obj(w.x)
        o.grad(w.x)
        o.cons(w.x)
        o.jac_coord(w.x)
        o.hess_coord(w.x, w.y, 1.0)
        o.jprod(w.x, v)
        o.jtprod(w.x, wv)
        o.hprod(w.x, w.y, 1.0, v)
        busy += time.perf_counter() - t0
        nnz += o.nnzj + o.nnzh
        n += 1
        i += workers
    return nnz, busy, n


def cpu_baseline(seconds):
    """The CPU oracle timed on the host's cores (before the GPU is used):
    one process, then one process per core (at most 16, the CPU share of
    one GPU on the measured boxes), each evaluating every callback of whole
    instances of the 256-instance workload.  nnz/s = Jacobian + Hessian
    entries of the instances done / wall time."""
    import concurrent.futures as cf
    import multiprocessing as mp
    nnz1, t1, n1 = _oracle_instances(0, 1, seconds)
    workers = max(1, min(os.cpu_count() or 1, 16))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        res = list(ex.map(_oracle_instances, range(workers), [workers] * workers, [seconds] * workers))
    wall = time.perf_counter() - t0
    nnzp = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    np_ = sum(r[2] for r in res)
    return dict(value=nnzp / busy, unit="nnz/s", cores=workers, kind="oracle",
                single_thread_value=nnz1 / t1, single_thread_cores=1,
                cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
                sample=(f"every callback (obj, grad, cons, jac, hess, jprod, jtprod, hprod) of whole instances of "
                        f"the 256-instance ACOPF batch (seeds 1000+): {n1} instances in {t1:.1f} s on one core; "
                        f"{np_} instances on {workers} processes, the longest busy {busy:.1f} s "
                        f"(wall {wall:.1f} s with setup); numpy float64, the oracle as it stands"))


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
    global QUICK, EVAL_SCHEDULE, BATCH_SCHEDULE
    args = parse()
    QUICK = args.quick
    EVAL_SCHEDULE = args.eval_schedule
    BATCH_SCHEDULE = args.batch_schedule
    if args.copy_mib:
        copy_only(args.copy_mib)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(instances of a batch would be sharded across GPUs with no exchange; not implemented).",
              file=sys.stderr)
        sys.exit(2)
    out = {"metric": METRIC, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    cpu = None
    if args.only in (None, "batch") and not args.no_cpu_baseline:
        # before anything touches the GPU: the worker processes are forked
        log("leg: cpu baseline")
        cpu = cpu_baseline(args.cpu_seconds)
        log(json.dumps(cpu))
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from exa_modeling.generators import acopf, pde

    if args.only in (None, "batch"):
        log("leg: batched 256 (headline)")
        r = leg_batch(args.steps, args.warmup)
        log(json.dumps(r))
        out.update(value=r["nnz_per_s"], ms_per_step=r["step_s"] * 1e3)
        out["config"] = {"workload": "acopf-batch-256: 256 uneven ACOPF instances, buses log-uniform in "
                                     "500-20,000 (1,399,478 in total), loads x U(0.9, 1.1), seeds 1000-1255",
                         "step": "exa_batch_eval of obj, grad, cons, jac, hess, jprod, jtprod, hprod for every "
                                 "instance at one iterate (one graph replay: evaluation launch + reduction launch)",
                         "instances": r["instances"], "buses": r["buses"], "nvar": r["nvar"], "ncon": r["ncon"],
                         "nnzj": r["nnzj"], "nnzh": r["nnzh"], "schedule": r["schedule"]}
        from exa_modeling.generators import acopf as _acopf
        traffic, tsched = profiled_traffic("batch256_eval_all.md", _acopf(30, 0).model, r["eval_kernel"])
        out["roofline"] = {"kernel": r["eval_kernel"], "bound": "hbm", "achieved": r["eval_gbs"],
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": r["eval_gbs"] / HBM_PEAK_GBS,
                           "traffic": traffic, "traffic_schedule": tsched, "bytes_per_launch": r["eval_bytes"],
                           "read_bytes": r["eval_read_bytes"], "write_bytes": r["eval_write_bytes"],
                           "launch_us": r["eval_us"], "launches_timed": r["launches_timed"]}
        out["roofline_reduce"] = {"kernel": "k_reduce_batch", "achieved": r["reduce_gbs"],
                                  "frac": (r["reduce_gbs"] or 0.0) / HBM_PEAK_GBS,
                                  "bytes_per_launch": r["reduce_bytes"], "launch_us": r["reduce_us"]}
        out["batched"] = {k: v for k, v in r.items() if k not in ("schedule",)}
        if cpu is not None:
            out["cpu_baseline"] = cpu
        cg = copy_gbs()
        out["hbm_copy_gbs"] = cg["exa_device_copy"]
        out["hbm_copy_torch_gbs"] = cg["torch"]
    if not args.no_extras and args.only in (None, "acopf"):
        log("leg: acopf 10k")
        wl = acopf(10000, 1)
        r = leg_single("acopf10k", wl, args.steps, args.warmup)
        log(json.dumps(r))
        traffic, tsched = profiled_traffic("acopf10k_eval_all.md", acopf(30, 0).model, r["eval_kernel"])
        out["acopf10k"] = {
            "workload": "acopf-10000-bus (13,500 branches, 2,000 generators, seed 1)",
            "step": "exa_eval of obj, grad, cons, jac, hess, jprod, jtprod, hprod at one iterate",
            "nvar": r["nvar"], "ncon": r["ncon"], "nnzj": r["nnzj"], "nnzh": r["nnzh"],
            "step_us": round(r["step_s"] * 1e6, 2), "nnz_per_s": r["nnz_per_s"], "schedule": r["schedule"],
            "step_separate_us": r["step_separate_us"], "step_graph_us": r["step_graph_us"],
            "rotated": r["rotated"], "callbacks_us": r["callbacks_us"],
            "jac_hess_nnz_per_s": r["jac_hess_nnz_per_s"], "ipm_step_us": r["ipm_step_us"],
            "ipm_nnz_per_s": r["ipm_nnz_per_s"], "jac_plus_hess_nnz_per_s": r["jac_plus_hess_nnz_per_s"],
            "roofline_eval": {"kernel": r["eval_kernel"], "achieved": r["eval_gbs"], "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": r["eval_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                              "traffic_schedule": tsched,
                              "bytes_per_launch": r["eval_bytes"], "launch_us": r["eval_us"]},
            "roofline_reduce": {"kernel": "k_reduce", "achieved": r["reduce_gbs"],
                                "bytes_per_launch": r["reduce_bytes"], "launch_us": r["reduce_us"]},
            "roofline_jac_hess_coord": {"kernel": "exa_k_jh", "achieved": r["jh_gbs"],
                                        "frac": r["jh_gbs"] / HBM_PEAK_GBS, "bytes_per_launch": r["jh_bytes"],
                                        "launch_us": r["jh_kernel_us"]}}
        if args.only == "acopf":
            out.update(value=r["nnz_per_s"], ms_per_step=r["step_s"] * 1e3)
    if not args.no_extras and args.only in (None, "pde"):
        log("leg: pde 1000")
        wl = pde(1000, 3)
        r = leg_single("pde1000", wl, max(20, args.steps // 20), 5)
        log(json.dumps(r))
        traffic, tsched = profiled_traffic("pde1000_eval_all.md", pde(8, 3).model, r["eval_kernel"])
        out["pde"] = {"workload": "pde-control 1000x1000 grid (2e6 variables, seed 3)",
                      "nnzj": r["nnzj"], "nnzh": r["nnzh"], "step_us": round(r["step_s"] * 1e6, 2),
                      "nnz_per_s": r["nnz_per_s"], "step_separate_us": r["step_separate_us"],
                      "step_graph_us": r["step_graph_us"], "schedule": r["schedule"],
                      "rotated": r["rotated"],
                      "jac_hess_nnz_per_s": r["jac_hess_nnz_per_s"],
                      "ipm_step_us": r["ipm_step_us"], "ipm_nnz_per_s": r["ipm_nnz_per_s"],
                      "callbacks_us": r["callbacks_us"],
                      "roofline_eval": {"kernel": r["eval_kernel"], "achieved": r["eval_gbs"],
                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": r["eval_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                                        "traffic_schedule": tsched,
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
