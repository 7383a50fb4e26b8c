#!/usr/bin/env python3
"""Throughput of the Q + Tw map on one MI355X.

One step = one fastqsl_q2d call on the 256x256x128 FP32 cube (6 seeded charges plus
an arched, uniformly twisted flux tube) with 1024 x 1024 seeds on z = 0: field
preparation, FP32 tracing of both halves of every line, the FP64 re-trace of
grazing lines, and the FP64 Q/Tw/length stencil. The field is resident in HBM
before the timed region. The headline times K such maps with --in-flight (4) of
them in flight on as many streams (the current one among them), each with its own
workspace, so that one map's
FP64 pass overlaps the next maps' FP32 passes; the same maps one at a time, and
the kernel timings the roofline takes, come from a run with one map in flight.
Prints ONE JSON line on stdout; details go to stderr.

  python bench.py [--steps K] [--warmup W] [--precision f32x|f64] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Q+Tw values/sec at 1 GPU (FP32+FP64-fixup vs all-FP64) at stated log10Q error"
UNIT = "Q+Tw values/s"

# Algorithmic FP operations of the method per Runge-Kutta stage (FMA = 2), as the
# method defines them and independent of this design: trilinear weights ~12, 2 x 3 x
# 7 lerps ~84, normalisation ~8, twist integrand ~8, stage combination ~18 = 130;
# six stages per RKF45 trial step = 780. (The design's own extra work, the monomial
# coefficients of each fetched cell and the landing logic, is not counted.)
FLOPS_PER_STAGE = 130
STAGES_PER_TRIAL = 6
FLOPS_PER_TRIAL = FLOPS_PER_STAGE * STAGES_PER_TRIAL
# Gathered bytes the method reads per stage: B and curl B at 8 corners, FP32 (the
# design fetches them once per cell visit instead, 192 B per fetch)
BYTES_PER_STAGE = 192
BYTES_PER_FETCH = 192
# MI355X vector FP32 without packed instructions (the library is built with packed
# FP32 switched off): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz; the
# published FP32 vector figure counts packed (two-wide) FP32 instructions.
PEAK_FP32_VECTOR = 256 * 4 * 16 * 2 * 2.4e9
PEAK_FP32_PUBLISHED = 157.3e12
# The paper's own GPU throughput for this path (Table 1: Method I, RKF45,
# tol_perp = 10^-3.2, on an RTX 3070 OC, TD99 flux-rope model): context, not a target
PAPER_GPU_Q_PER_S = 4.53e6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """HIP events from the runtime torch has loaded (for timing one kernel)."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, n):
        arr = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            rc = self.lib.hipEventCreate(ctypes.byref(h))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed: {rc}")
            arr[i] = h
        return arr

    def ms(self, a, b) -> float:
        out = ctypes.c_float()
        rc = self.lib.hipEventElapsedTime(ctypes.byref(out), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(out.value)


def traffic_from_profile(workload: str, prec: str):
    """HBM bytes per launch of the tracer from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "trace_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(f"{workload}/{prec}")
        from paper_2208_12569_amd.profiling import kernel_source_sha

        if e and e.get("kernel_source_sha") == kernel_source_sha():
            return float(e["traffic_bytes_per_launch"])
    except (ValueError, KeyError):
        return None
    return None


def run_gpu(w, prec_name: str, tol: float, steps: int, warmup: int, method: int = 0):
    import torch

    import paper_2208_12569_amd as fq

    prec = fq.FQ_PREC_F64 if prec_name == "f64" else fq.FQ_PREC_F32X
    mk = {"method": method}
    B = torch.from_numpy(w.field).cuda()
    torch.cuda.synchronize()
    stats = torch.zeros(5, dtype=torch.int64, device="cuda")
    ev = HipEvents()
    ws = None
    first_ms = None
    for _ in range(max(1, warmup)):
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        r = fq.q2d(B, w.grid, w.plane, fq.Params(precision=prec, tol_perp=tol, **mk), ws=ws)
        c1.record()
        c1.synchronize()
        if first_ms is None:
            first_ms = c0.elapsed_time(c1)  # cold: first call of the process
        ws = r["_ws"]
    torch.cuda.synchronize()
    evs = [ev.create(4) for _ in range(steps)]
    # one event between consecutive calls: per-call times for the median
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    marks[0].record()
    for k in range(steps):
        r = fq.q2d(B, w.grid, w.plane,
                   fq.Params(precision=prec, tol_perp=tol, stats=stats, events=evs[k], **mk), ws=ws)
        marks[k + 1].record()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    call_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    median_ms = (call_ms[(steps - 1) // 2] + call_ms[steps // 2]) / 2.0
    trace_ms = [ev.ms(e[0], e[1]) for e in evs]
    fix_ms = [ev.ms(e[2], e[3]) for e in evs] if prec == fq.FQ_PREC_F32X else [0.0] * steps
    st = [int(x) // steps for x in stats.tolist()]
    # the FP32 pass alone (the same pass without the FP64 re-trace after it), for the
    # per-kernel counts of the roofline
    st32 = st
    if prec == fq.FQ_PREC_F32X:
        s32 = torch.zeros(5, dtype=torch.int64, device="cuda")
        fq.q2d(B, w.grid, w.plane, fq.Params(precision=prec, tol_perp=tol, graze=-1.0, stats=s32, **mk),
               ws=ws)
        torch.cuda.synchronize()
        st32 = [int(x) for x in s32.tolist()]
    q = r["q"]
    status = r["status"]
    fatal = int(((status.to(torch.int32) & fq.ST_FATAL) != 0).sum())
    finite = int(torch.isfinite(q).sum())
    log(f"[{prec_name}] {steps} steps: {total_ms / steps:.3f} ms/step (wall {wall * 1e3 / steps:.3f}), "
        f"tracer {sum(trace_ms) / steps:.3f} ms, FP64 pass {sum(fix_ms) / steps:.3f} ms; per step: "
        f"trials {st[0]}, accepted {st[1]}, fetches {st[2]}, halves {st[3]}, FP64 halves {st[4]}; "
        f"finite Q {finite}, fatal {fatal}")
    return {"ms": total_ms / steps, "median_ms": median_ms, "trace_ms": sum(trace_ms) / steps,
            "fix_ms": sum(fix_ms) / steps, "stats": st, "stats32": st32, "first_ms": first_ms,
            "map": {"q": r["q"].cpu().numpy(), "tw": r["tw"].cpu().numpy(),
                    "status": r["status"].cpu().numpy().astype("uint16"),
                    **({"qperp": r["qperp"].cpu().numpy()} if "qperp" in r else {})},
            "params": fq.Params(precision=prec, tol_perp=tol, **mk)}


_SIDE_STREAMS: list = []


def run_in_flight(w, prec_name: str, tol: float, steps: int, warmup: int, n: int = 4):
    """The same maps with n of them in flight at once, on n streams of default priority
    (the current stream and n - 1 more: the GPU runs four hardware queues, and a fifth
    stream would share one) with a workspace each: one map's FP64 pass and stencil (a
    tail that leaves most SIMDs idle) overlap the next maps' FP32 passes. Every map is
    computed whole; they are checked equal, bit for bit, to the same map computed
    alone."""
    import torch

    import paper_2208_12569_amd as fq

    prec = fq.FQ_PREC_F64 if prec_name == "f64" else fq.FQ_PREC_F32X
    B = torch.from_numpy(w.field).cuda()
    # in_flight: the F32X form's FP64 pass at three waves per SIMD, leaving room for
    # the other maps' FP32 waves (same results)
    p = fq.Params(precision=prec, tol_perp=tol, in_flight=True)
    # the side streams are made once per process: HIP assigns hardware queues to
    # streams in the order they are created, and new ones for every run would come to
    # share a queue with the current stream
    while len(_SIDE_STREAMS) < n - 1:
        _SIDE_STREAMS.append(torch.cuda.Stream())
    streams = [torch.cuda.current_stream()] + _SIDE_STREAMS[:n - 1]
    wss = []
    for s in streams:
        with torch.cuda.stream(s):
            wss.append(fq.q2d(B, w.grid, w.plane, p, stream=s)["_ws"])
    torch.cuda.synchronize()
    for k in range(max(1, warmup) * n):
        s = streams[k % n]
        with torch.cuda.stream(s):
            fq.q2d(B, w.grid, w.plane, p, stream=s, ws=wss[k % n])
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(main)
    for s in streams:
        s.wait_event(t0)
    outs = []
    for k in range(steps):
        s = streams[k % n]
        with torch.cuda.stream(s):
            outs.append(fq.q2d(B, w.grid, w.plane, p, stream=s, ws=wss[k % n])["q"])
    for s in streams:
        e = torch.cuda.Event()
        e.record(s)
        main.wait_event(e)
    t1.record(main)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1) / steps
    # every map equals the first, and the first the map one at a time (no in_flight)
    one = fq.q2d(B, w.grid, w.plane, fq.Params(precision=prec, tol_perp=tol))["q"]
    torch.cuda.synchronize()
    ref = one.nan_to_num(-1.0)
    same = all(bool(torch.equal(o.nan_to_num(-1.0), ref)) for o in outs)
    log(f"[{prec_name}] {steps} steps, {n} maps in flight: {ms:.3f} ms/step "
        f"(wall {wall * 1e3 / steps:.3f}); maps identical: {same}")
    if not same:
        raise RuntimeError("maps computed in flight on several streams differ")
    return {"ms": ms, "wall_ms": wall * 1e3 / steps, "streams": n}


def sampled_accuracy(w, gmaps: dict, k: int = 3000, seed: int = 7, method: int = 0) -> dict:
    """The oracle (FP64, tol 1e-10) at k interior map points drawn at random against
    each form's map: Method I through each point's own stencil (q2d_points), Method
    II through its own line (method2, offset differences of B/B), Q_perp too."""
    import numpy as np

    import oracle

    pl = w.plane
    rng = np.random.default_rng(seed)
    ii = rng.integers(1, pl.nu - 1, k)
    jj = rng.integers(1, pl.nv - 1, k)
    idx = np.unique(jj * pl.nu + ii)
    t = time.perf_counter()
    if method == 1:
        o = oracle.method2(w.field, w.grid, pl.points()[idx], 2, {"tol": 1e-10})
    else:
        o = oracle.q2d_points(w.field, w.grid, pl, idx, {"tol": 1e-10})
    dt = time.perf_counter() - t
    res = {"sample": f"{idx.size} interior map points drawn at random",
           "oracle_values_per_s": idx.size / dt, "oracle_cores": oracle.threads()}
    for form, g in gmaps.items():
        res[form] = err_stats(g["q"].ravel()[idx], g["tw"].ravel()[idx], g["status"].ravel()[idx],
                              np.asarray(o["q"]).ravel(), np.asarray(o["tw"]).ravel(),
                              np.asarray(o["status"]).ravel())
        if method == 1:
            qp = err_stats(g["qperp"].ravel()[idx], g["tw"].ravel()[idx], g["status"].ravel()[idx],
                           np.asarray(o["qperp"]).ravel(), np.asarray(o["tw"]).ravel(),
                           np.asarray(o["status"]).ravel())
            res[form]["qperp_logq_rel_max"] = qp["logq_rel_max"]
            res[form]["qperp_points_over_1e-4"] = qp["points_over_1e-4"]
    return res


def run_variant(w, label: str, args, uniform_value: float, method: int = 0) -> dict:
    """One more workload in both forms, with its sampled accuracy: the stretched C2
    grid, or Method II on C2."""
    npts = w.plane.nu * w.plane.nv
    out = {"workload": label, "unit": UNIT}
    maps = {}
    for form in ("f32x", "f64"):
        r = run_gpu(w, form, args.tol, args.sub_steps, args.warmup, method=method)
        out[form] = {"value": npts / (r["ms"] * 1e-3), "ms_per_step": r["ms"], "trace_ms": r["trace_ms"],
                     "fp64_pass_ms": r["fix_ms"], "trial_steps": r["stats"][0],
                     "vs_uniform_method1": npts / (r["ms"] * 1e-3) / uniform_value[form]}
        maps[form] = r["map"]
    if not args.no_cpu_baseline:
        out["accuracy"] = sampled_accuracy(w, maps, method=method)
    log(f"{label}: {out}")
    return out


def gather_roofline(nodes: int, nx: int, ny: int, nz: int, walk_steps: int = 400):
    """Sustained rate of the tracer's cell fetches (8 corner records of B and curl B,
    16 vector loads) along field-line-like walks with no arithmetic, on a record
    array of the same size and layout; the best over 1-4 resident blocks per CU, for
    incoherent walks (each lane its own moves) and coherent ones (the lanes of a wave
    on an 8 x 8 patch of cells, taking the same moves). Returns (coherent, incoherent)
    rates in useful bytes per second."""
    import torch

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2208_12569_amd", "libfqgather.so"))
    lib.fqgb_walk.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_void_p]
    rec = torch.rand((nodes, 8), dtype=torch.float32, device="cuda")
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    out = []
    for coherent in (1, 0):
        best = 0.0
        rates = {}
        for per_cu in (1, 2, 3, 4):
            blocks = ncu * per_cu
            sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
            stream = torch.cuda.current_stream().cuda_stream
            rc = lib.fqgb_walk(rec.data_ptr(), nx, ny, nz, walk_steps, blocks, 1, coherent,
                               sink.data_ptr(), stream)
            if rc != 0:
                raise RuntimeError(f"gather microbenchmark launch failed: {rc}")
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            lib.fqgb_walk(rec.data_ptr(), nx, ny, nz, walk_steps, blocks, 2, coherent,
                          sink.data_ptr(), stream)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b)
            rate = blocks * 256 * walk_steps * 192 / (ms * 1e-3)
            rates[per_cu * 4] = rate / 1e9
            best = max(best, rate)
        log(f"gather microbenchmark, {'coherent' if coherent else 'incoherent'} walks (GB/s of useful "
            "gathered bytes by resident waves per CU): " + ", ".join(f"{k}: {v:.0f}" for k, v in rates.items()))
        out.append(best)
    return out[0], out[1]


def valu_fma_rate(iters: int = 20000):
    """Sustained FP32 FMA rate of the chip's vector units (unpacked, as the library
    is built): 8 independent FMA chains per lane, the best over 1-8 resident blocks
    per CU. Returns FLOP/s."""
    import torch

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2208_12569_amd", "libfqgather.so"))
    lib.fqgb_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    stream = torch.cuda.current_stream().cuda_stream
    best = 0.0
    rates = {}
    for per_cu in (1, 2, 4, 8):
        blocks = ncu * per_cu
        sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
        if lib.fqgb_fma(iters, blocks, sink.data_ptr(), stream) != 0:
            raise RuntimeError("FMA microbenchmark launch failed")
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        lib.fqgb_fma(iters, blocks, sink.data_ptr(), stream)
        b.record()
        b.synchronize()
        rate = blocks * 256 * iters * 16 / (a.elapsed_time(b) * 1e-3)
        rates[per_cu * 4] = rate / 1e12
        best = max(best, rate)
    log("FP32 FMA microbenchmark (TFLOP/s by resident waves per CU): "
        + ", ".join(f"{k}: {v:.1f}" for k, v in rates.items()))
    return best


def run_batch(seed: int, steps: int, warmup: int):
    """The uneven batch: 16 seeded cubes (edges 64-384, FP32, 4-12 charges, seed grids
    128^2-1024^2 on z = 0) in one persistent launch, captured in a HIP graph with
    autotuned launch parameters; against the same jobs run one call each."""
    import torch

    import paper_2208_12569_amd as fq
    from paper_2208_12569_amd.graph import Q2DGraph
    from paper_2208_12569_amd.tune import tune_launch
    from synth.torch_fields import config_c4_torch

    t = time.perf_counter()
    ws_ = config_c4_torch(seed)
    jobs = [(w.field, w.grid, w.plane) for w in ws_]
    torch.cuda.synchronize()
    log(f"generated the 16-cube batch on the GPU in {time.perf_counter() - t:.1f} s")
    npts = sum(w.plane.nu * w.plane.nv for w in ws_)
    params, table = tune_launch(jobs, fq.Params(), reps=2)
    log(f"batch tuner: block {params.block}, waves/CU {params.waves_per_cu}; "
        + ", ".join(f"{k}: {v:.2f} ms" for k, v in sorted(table.items())))
    g = Q2DGraph(jobs, params)
    for _ in range(max(1, warmup)):
        g.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    # each job alone: one call per job, same parameters, median of 3
    alone = 0.0
    for j in jobs:
        need = fq.q2d_workspace_size([j], params)
        wsb = torch.empty(need, dtype=torch.uint8, device="cuda")
        outs = fq.alloc_q2d_outputs([j])
        fq.q2d_batch_into([j], outs, wsb, params)
        tt = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fq.q2d_batch_into([j], outs, wsb, params)
            e1.record()
            e1.synchronize()
            tt.append(e0.elapsed_time(e1))
        alone += sorted(tt)[1]
        del wsb, outs
    # two instances of the captured batch (their own workspaces and outputs) replayed
    # in flight on two streams: one batch's FP64 pass overlaps the other's FP32 pass
    import dataclasses

    pf = dataclasses.replace(params, in_flight=True)
    ga, gb2 = Q2DGraph(jobs, pf), Q2DGraph(jobs, pf)
    while len(_SIDE_STREAMS) < 1:
        _SIDE_STREAMS.append(torch.cuda.Stream())
    side, main = _SIDE_STREAMS[0], torch.cuda.current_stream()

    def pair(k):
        if k % 2 == 0:
            ga.replay()
        else:
            with torch.cuda.stream(side):
                gb2.replay()

    for k in range(2 * max(1, warmup)):
        pair(k)
    torch.cuda.synchronize()
    a.record(main)
    side.wait_event(a)
    for k in range(steps):
        pair(k)
    e_side = torch.cuda.Event()
    e_side.record(side)
    main.wait_event(e_side)
    b.record(main)
    torch.cuda.synchronize()
    graphs_ms = a.elapsed_time(b) / steps
    del ga, gb2
    # the same jobs as single calls, four in flight (q2d_many), for comparison
    for _ in range(max(1, warmup)):
        fq.q2d_many(jobs, params)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        fq.q2d_many(jobs, params)
    b.record()
    torch.cuda.synchronize()
    many_ms = a.elapsed_time(b) / steps
    log(f"[batch] {ms:.3f} ms per graph replay of 16 jobs ({npts} values); one call per job: "
        f"{alone:.3f} ms; one call per job, four in flight: {many_ms:.3f} ms; two graph replays "
        f"in flight: {graphs_ms:.3f} ms per batch")
    return {"workload": "16 seeded cubes, edges U{64..384} (FP32, 4-12 charges), seed grids "
                        "U{128,256,512,1024}^2 on z=0, one persistent launch in a HIP graph",
            "value": npts / (ms * 1e-3), "unit": UNIT, "ms_per_batch": ms, "values": npts,
            "one_call_per_job_ms": alone, "batching_gain": alone / ms,
            "one_call_per_job_four_in_flight_ms": many_ms,
            "two_graph_replays_in_flight_ms_per_batch": graphs_ms,
            "params": {"block": params.block, "waves_per_cu": params.waves_per_cu}}


def run_adjoint(seed: int, steps: int, warmup: int, prec_name: str = "f64"):
    """The adjoint workload: the 256x256 map of a 128x128x96 FP32 cube from 8 point
    charges, and the gradient of a log10 Q + footpoint loss against a target map
    with respect to the node values (all-FP64 form, or the F32X form whose FP32 pass
    is replayed and reversed in FP32; checkpoints every 32 accepted steps): per step,
    the map traced once with its checkpoints kept (fastqsl_q2d_record), the loss,
    and the reverse pass (fastqsl_backward_recorded)."""
    import torch

    import paper_2208_12569_amd as fq
    import synth
    from synth.torch_fields import charges_field_torch

    w, target = synth.config_c5(seed)
    g, pl = w.grid, w.plane
    pos, q = w.meta["charges"]
    B = charges_field_torch(g, pos, q, torch.float32, "cuda")
    tB = charges_field_torch(g, *target["charges"], torch.float32, "cuda")
    prec = fq.FQ_PREC_F64 if prec_name == "f64" else fq.FQ_PREC_F32X
    p = fq.Params(precision=prec)
    tq = fq.q2d(tB, g, pl, fq.Params(precision=fq.FQ_PREC_F64))["q"]
    stats = torch.zeros(5, dtype=torch.int64, device="cuda")
    gb = torch.zeros(B.shape, dtype=torch.float64, device="cuda")
    ws = [None]  # the record's workspace, reused from step to step

    def step(st=None):
        r = fq.q2d_record(B, g, pl, p, 32, ws=ws[0])
        ws[0] = r["_ws"]
        qq = r["q"]
        m = torch.isfinite(qq) & torch.isfinite(tq) & (qq < 1e8) & (tq < 1e8)
        lq = torch.log10(torch.where(m, qq, torch.ones_like(qq)))
        lt = torch.log10(torch.where(m, tq, torch.ones_like(tq)))
        dq = torch.where(m, 2.0 * (lq - lt) / (qq * math.log(10.0)), torch.zeros_like(qq)) / m.sum()
        gb.zero_()
        fq.backward_recorded(B, g, pl, r, fq.Params(precision=prec, stats=st), 32,
                             dq=dq.reshape(-1), gb=gb)

    for _ in range(max(1, warmup)):
        step()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step(stats)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    st = [int(x) // steps for x in stats.tolist()]
    npts = pl.nu * pl.nv
    log(f"[adjoint {prec_name}] {ms:.3f} ms per map + gradient; half lines differentiated {st[0]}, "
        f"accepted steps reversed {st[1]}, replay mismatches {st[2]}")
    form = "FP64" if prec_name == "f64" else "F32X: FP32 pass, replay and reverse sweep"
    return {"workload": "128x128x96 FP32 cube, 8 point charges, 256x256 seeds on z=0; forward "
                        "map traced once with checkpoints + dL/dB of a log10 Q loss vs a target "
                        f"map ({form}, checkpoint every 32 accepted steps)",
            "value": npts / (ms * 1e-3), "unit": "map points with gradient/s", "ms_per_step": ms,
            "half_lines": st[0], "steps_reversed": st[1], "replay_mismatches": st[2]}


def cpu_baseline(w, side: int):
    """The oracle on a bounded sample: a side x side block of the same seed grid
    (centre of the map), traced and assembled on the host cores."""
    import numpy as np

    import oracle
    import synth

    pl = w.plane
    i0 = (pl.nu - side) // 2
    j0 = (pl.nv - side) // 2
    o = np.asarray(pl.origin) + i0 * pl.du * np.asarray(pl.u) + j0 * pl.dv * np.asarray(pl.v)
    sub = synth.Plane(tuple(o), pl.u, pl.v, side, side, pl.du, pl.dv)
    oracle.build()
    t = time.perf_counter()
    r = oracle.q2d(w.field, w.grid, sub, {"tol": 1e-10}, want_lines=True)
    dt = time.perf_counter() - t
    n = side * side
    return {"value": n / dt, "unit": UNIT, "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{side}x{side} block at the centre of the 1024x1024 seed grid (same cube, "
                      f"oracle tol 1e-10 grid spacings); {dt:.1f} s incl. curl",
            "finite_q": int(np.isfinite(r["q"]).sum()), "_map": r, "_at": (i0, j0, side)}


def cpu_c1_rows() -> dict:
    """The oracle on the full 128 x 128 map of the 4-charge 64^3 FP64 cube on the host
    cores, at its parity tolerance (1e-10 grid spacings) and at the paper's marginal
    RKF45 tolerance 10^-3.2 (Table 1), for comparison with the paper's CPU rows.
    The oracle always integrates cell by cell and lands on faces; only its error
    bound changes."""
    import oracle
    import synth

    w = synth.config_c1(0)
    out = {}
    for name, tol in (("tol_1e-10", 1e-10), ("tol_10^-3.2", 10 ** -3.2)):
        t = time.perf_counter()
        oracle.q2d(w.field, w.grid, w.plane, {"tol": tol}, want_lines=False)
        dt = time.perf_counter() - t
        out[name] = {"value": w.plane.nu * w.plane.nv / dt, "unit": "Q+Tw values/s",
                     "seconds": dt}
    out["cores"] = oracle.threads()
    out["workload"] = "64^3 FP64 cube, 4 seeded charges, 128x128 seeds on z=0 (full map)"
    return out


def err_stats(qg, twg, sg, qo, two, so) -> dict:
    """Errors of GPU values against the oracle's on the points where both succeed, no
    stencil line ends near a box edge and Q < 1e8: relative error of log10 Q on the
    scale max(|log10 Q|, log10 2) (max, 99.9th percentile, count over 1e-4), and the
    absolute error of Tw."""
    import numpy as np

    import paper_2208_12569_amd as fq

    sg = sg.astype(np.uint16)
    so = so.astype(np.uint16)
    bad = fq.ST_FATAL | fq.ST_MIXEDFACE | fq.ST_EDGE
    m = (((sg | so) & bad) == 0) & np.isfinite(qo) & np.isfinite(qg) & (qo < 1e8)
    lo = np.log10(np.where(m, qo, 1.0))
    lg = np.log10(np.where(m, qg, 1.0))
    rel = np.where(m, np.abs(lg - lo) / np.maximum(np.abs(lo), np.log10(2.0)), 0.0)
    tw_ok = (((sg | so) & fq.ST_FATAL) == 0) & np.isfinite(two) & np.isfinite(twg)
    out = {"points": int(m.sum()), "logq_rel_max": float(rel[m].max()),
           "logq_rel_p999": float(np.quantile(rel[m], 0.999)),
           "points_over_1e-4": int((rel > 1e-4).sum()),
           "tw_abs_max": float(np.abs(twg[tw_ok] - two[tw_ok]).max())}
    return out


def block_ends(w, params, at):
    """End points of both halves of every line of the oracle's block, from one more
    call of the timed form (the timed runs keep no lines)."""
    import numpy as np
    import torch

    import paper_2208_12569_amd as fq

    i0, j0, side = at
    B = torch.from_numpy(w.field).cuda()
    r = fq.q2d(B, w.grid, w.plane, params, want_lines=True)
    torch.cuda.synchronize()
    out = {}
    for k in ("end_b", "end_f"):
        e = r["lines"][k].reshape(w.plane.nv, w.plane.nu, 3)[j0:j0 + side, i0:i0 + side]
        out[k] = e.cpu().numpy().reshape(-1, 3)
    return out


def foot_stats(ends: dict, orc: dict, side: int) -> dict:
    """Footpoint errors (box units, max over both ends of a line) on the block's
    interior, against the bound 1e-6 where Q < 1e4 and 1e-6 sqrt(Q/1e4) above (the map
    stretches a line's error by about sqrt(Q))."""
    import numpy as np

    import paper_2208_12569_amd as fq

    d = np.zeros(side * side)
    for k in ("end_b", "end_f"):
        d = np.maximum(d, np.abs(ends[k] - orc["lines"][k]).max(axis=1))
    qo = orc["q"].ravel()
    st = orc["status"].ravel().astype(np.uint16)
    keep = ((st & (fq.ST_FATAL | fq.ST_EDGE)) == 0) & np.isfinite(qo) & (qo < 1e8)
    inner = np.zeros((side, side), bool)
    inner[1:-1, 1:-1] = True
    keep &= inner.ravel() & np.isfinite(d)
    bound = 1e-6 * np.maximum(1.0, np.sqrt(qo / 1e4))
    return {"foot_max": float(d[keep].max()), "foot_over_bound": int((d[keep] > bound[keep]).sum()),
            "foot_max_over_bound": float((d[keep] / bound[keep]).max())}


def accuracy(gmap: dict, orc: dict, at, w) -> dict:
    """Errors of a GPU map against the oracle on the oracle's block, away from the
    block's border (where the block's own stencil is one-sided), on the parity mask
    of the tests (both sides succeed, no stencil line ends near a box edge,
    Q < 1e8)."""
    i0, j0, side = at
    sl = (slice(j0 + 1, j0 + side - 1), slice(i0 + 1, i0 + side - 1))
    r = err_stats(gmap["q"][sl], gmap["tw"][sl], gmap["status"][sl],
                  orc["q"].reshape(side, side)[1:-1, 1:-1],
                  orc["tw"].reshape(side, side)[1:-1, 1:-1],
                  orc["status"].reshape(side, side)[1:-1, 1:-1])
    r["against"] = "the oracle (FP64, tol 1e-10) on the CPU-baseline block"
    return r


def run_q3d(seed: int, steps: int, warmup: int, sample: int = 3000):
    """The 3-D map: Q, Tw and length at the 256x256x128 voxel centres of the
    512x512x256 FP32 cube (10 seeded charges, two arched tubes of opposite
    handedness). Voxels where |Bz/B| < 0.05 turn S0 perpendicular to B and trace 4
    extra lines. Both forms: the first call and the mean of `steps` warm calls.
    Keeps the values at sampled voxels (random ones and rotated ones) for the
    oracle comparison of the CPU-baseline leg."""
    import numpy as np
    import torch

    import paper_2208_12569_amd as fq
    from synth.torch_fields import config_c3_torch

    t = time.perf_counter()
    w = config_c3_torch(seed)
    torch.cuda.synchronize()
    log(f"generated {w.name} on the GPU in {time.perf_counter() - t:.1f} s")
    vx = w.voxels
    n = int(np.prod(vx.n))
    out = {"workload": "512x512x256 FP32 cube (dx=1/511), 10 seeded charges + 2 arched tubes "
                       "(1.5 turns, opposite handedness); Q, Tw, length at 256x256x128 voxel "
                       "centres, S0 turned perpendicular to B where |Bz/B| < 0.05",
           "unit": UNIT, "voxels": n}
    keep = {}
    for name, prec in (("f32x", fq.FQ_PREC_F32X), ("f64", fq.FQ_PREC_F64)):
        p = fq.Params(precision=prec)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        r = fq.q3d(w.field, w.grid, vx, p)
        c1.record()
        c1.synchronize()
        first = c0.elapsed_time(c1)
        ws = r["_ws"]
        for _ in range(max(0, warmup - 1)):
            r = fq.q3d(w.field, w.grid, vx, p, ws=ws)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            r = fq.q3d(w.field, w.grid, vx, p, ws=ws)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[name] = {"value": n / (ms * 1e-3), "ms_per_map": ms, "first_call_ms": first}
        keep[name] = {k: r[k].cpu().numpy().ravel() for k in ("q", "tw", "status")}
        if name == "f32x":
            # the FP32 pass alone (no FP64 pass), timed on its own stream with HIP
            # events, and its cell fetches: the tracer's gathered bytes per second
            ev = HipEvents()
            e4 = ev.create(4)
            s32 = torch.zeros(5, dtype=torch.int64, device="cuda")
            fq.q3d(w.field, w.grid, vx, fq.Params(precision=prec, graze=-1.0, stats=s32, events=e4),
                   ws=ws)
            torch.cuda.synchronize()
            tms = ev.ms(e4[0], e4[1])
            fetches = int(s32[2])
            out[name]["fp32_pass"] = {"trace_ms": tms, "cell_fetches": fetches,
                                      "gathered_GB_per_s": fetches * BYTES_PER_FETCH / (tms * 1e-3) / 1e9}
        log(f"[q3d {name}] {ms:.3f} ms per map (first call {first:.3f} ms)")
        del ws, r
    st = keep["f32x"]["status"].astype(np.uint16)
    rot = np.flatnonzero(st & fq.ST_ROTATED)
    out["rotated_voxels"] = int(rot.size)
    out["rotated_fraction"] = rot.size / n
    out["lines_traced"] = n + 4 * int(rot.size)
    rng = np.random.default_rng(29)
    idx = np.unique(np.concatenate([rng.choice(n, sample, replace=False),
                                    rng.choice(rot, min(sample // 10, rot.size), replace=False)]))
    out["_sample"] = (w, idx, {k: {c: v[idx] for c, v in d.items()} for k, d in keep.items()})
    return out


def q3d_accuracy(w, idx, gvals) -> dict:
    """The oracle at the sampled voxels (FP64, tol 1e-10 grid spacings) against both
    forms, and the oracle's rate on that sample."""
    import numpy as np

    import oracle

    Bh = w.field.cpu().numpy()
    t = time.perf_counter()
    o = oracle.q3d_points(Bh, w.grid, w.voxels, idx, {"tol": 1e-10})
    dt = time.perf_counter() - t
    import paper_2208_12569_amd as fq

    nrot = int(((gvals["f32x"]["status"].astype(np.uint16) & fq.ST_ROTATED) != 0).sum())
    res = {"sample": f"{idx.size} voxels drawn at random, plus rotated-S0 voxels drawn apart "
                     f"({nrot} rotated in all)",
           "oracle_values_per_s": idx.size / dt, "oracle_cores": oracle.threads()}
    for k, g in gvals.items():
        res[k] = err_stats(g["q"], g["tw"], g["status"], np.asarray(o["q"]).ravel(),
                           np.asarray(o["tw"]).ravel(), np.asarray(o["status"]).ravel())
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32,
                    help="timed maps of the headline workload (both forms)")
    ap.add_argument("--sub-steps", type=int, default=10,
                    help="timed steps of every other run (seeds, variants, batch, adjoint, 3-D map)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=("f32x", "f64"), default="f32x")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--in-flight", type=int, default=4,
                    help="maps in flight on as many streams for the headline throughput "
                         "(1: one map at a time)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true", help="skip the all-FP64 comparison run")
    ap.add_argument("--cpu-side", type=int, default=512)
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-cube batch run")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint run")
    ap.add_argument("--no-q3d", action="store_true", help="skip the 3-D map run")
    ap.add_argument("--no-seeds", action="store_true",
                    help="skip the runs of the same workload drawn with the two other seeds")
    ap.add_argument("--calib-copy", action="store_true",
                    help="finish with one 1 GiB device copy (calibrates rocprofv3 byte counters)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the stretched-grid and Method II runs of the C2 workload")
    ap.add_argument("--q3d-only", action="store_true",
                    help="run only the 3-D map of the 512x512x256 cube (for profiling it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this tracer runs on ONE GPU (no multi-GPU path is built); "
              "run with --gpus 1 — the value is that GPU's throughput", file=sys.stderr)
        sys.exit(2)

    import synth

    if args.q3d_only:
        r = run_q3d(args.seed, args.sub_steps, args.warmup)
        r.pop("_sample")
        if args.calib_copy:
            import torch

            x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
            y = torch.empty_like(x)
            y.copy_(x)
            torch.cuda.synchronize()
        print(json.dumps({"q3d": r}), flush=True)
        return

    t = time.perf_counter()
    w = synth.config_c2(args.seed)
    log(f"generated {w.name} in {time.perf_counter() - t:.1f} s")
    main_run = run_gpu(w, args.precision, args.tol, args.steps, args.warmup)
    nfl = max(1, args.in_flight)
    flight = run_in_flight(w, args.precision, args.tol, args.steps, args.warmup, nfl) if nfl > 1 else None
    other = other_flight = None
    if not args.no_f64 and args.precision == "f32x":
        other = run_gpu(w, "f64", args.tol, args.steps, args.warmup)
        if nfl > 1:
            other_flight = run_in_flight(w, "f64", args.tol, args.steps, args.warmup, nfl)

    npts = w.plane.nu * w.plane.nv
    # one map at a time (the latency of a map) and, the headline, several in flight
    seq_value = npts / (main_run["ms"] * 1e-3)
    step_ms = flight["ms"] if flight else main_run["ms"]
    value = npts / (step_ms * 1e-3)
    st = main_run["stats"]
    s32 = main_run["stats32"]
    # the method's flops: six stages per Runge-Kutta trial step (trial steps that end
    # a half line at a box face take no Runge-Kutta step)
    rk_trials = s32[0] - s32[3]
    flops = rk_trials * FLOPS_PER_TRIAL
    achieved = flops / (main_run["trace_ms"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32x" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "256x256x128 FP32 cube (dx=1/255), 6 seeded charges + arched twisted tube "
                        "(1.5 turns, radius 0.08); 1024x1024 cell-centred seeds on z=0; Q, Tw, length",
            "seed": args.seed,
            "precision": args.precision,
            "tol_perp": args.tol,
            "maps_in_flight": nfl,
            "one_map_at_a_time": {"value": seq_value, "ms_per_step": main_run["ms"],
                                  "median_ms_per_step": main_run["median_ms"]},
            "trace_ms": main_run["trace_ms"],
            "fp64_pass_ms": main_run["fix_ms"],
            "first_call_ms": main_run["first_ms"],
            "median_ms_per_step": main_run["median_ms"],
            "per_step": {"trial_steps": st[0], "accepted_steps": st[1], "cell_fetches": st[2],
                         "half_lines": st[3], "fp64_half_lines": st[4]},
            "fp32_pass": {"trial_steps": s32[0], "accepted_steps": s32[1], "cell_fetches": s32[2]},
        },
        "roofline": {
            "bound": "alu",
            "kernel": "trace_kernel<float, float, 1, true, false, 0, false> (FP32 pass)",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR,
            "traffic": traffic_from_profile("c2", args.precision),
            "flops_per_launch": flops,
            "counting": f"{FLOPS_PER_STAGE} method flops per Runge-Kutta stage x "
                        f"{STAGES_PER_TRIAL} stages x {rk_trials} trial steps per launch; peak = "
                        "256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz without packed FP32 "
                        "(which the build switches off)",
            "peak_published": PEAK_FP32_PUBLISHED / 1e12,
            "frac_of_published": achieved / PEAK_FP32_PUBLISHED,
        },
        "paper_context": {"value": PAPER_GPU_Q_PER_S, "unit": "Q values/s",
                          "hardware": "NVIDIA RTX 3070 OC", "workload": "TD99 flux-rope model, "
                          "Method I, RKF45, tol_perp = 10^-3.2 (Table 1)",
                          "note": "another machine, workload and accuracy; context, not the target"},
    }
    # the gather roofline: algorithmic gathered bytes of the tracer (192 B of B and
    # curl B per cell fetch) per second, against the microbenchmark's sustained rate
    g = w.grid
    micro, micro_inc = gather_roofline(g.nx * g.ny * g.nz, g.nx, g.ny, g.nz)
    # the same walks on record arrays of the other workloads' sizes: L2-resident
    # (64^3, 8.4 MB of records), the MALL-sized C2 above (268 MB), HBM-spilling
    # (512x512x256, 2.1 GB)
    by_size = {"256x256x128 (C2)": {"coherent": micro / 1e9, "incoherent": micro_inc / 1e9}}
    for label, (ax, ay, az) in (("64^3 (C1)", (64, 64, 64)), ("512x512x256 (C3)", (512, 512, 256))):
        c, i = gather_roofline(ax * ay * az, ax, ay, az)
        by_size[label] = {"coherent": c / 1e9, "incoherent": i / 1e9}
    gathered = s32[2] * BYTES_PER_FETCH / (main_run["trace_ms"] * 1e-3)
    per_stage = rk_trials * STAGES_PER_TRIAL * BYTES_PER_STAGE / (main_run["trace_ms"] * 1e-3)
    out["gather_roofline"] = {"achieved": gathered / 1e9, "peak": micro / 1e9, "unit": "GB/s",
                              "frac": gathered / micro, "incoherent_walks": micro_inc / 1e9,
                              "microbenchmark_by_record_array": by_size,
                              "method_bytes_per_stage_rate": per_stage / 1e9,
                              "note": "cell fetches x 192 B / tracer time, against the same "
                                      "fetches along field-line-like walks with no arithmetic "
                                      "whose 64 lanes per wave move together (neighbouring "
                                      "lines); walks whose lanes move apart reach "
                                      "incoherent_walks. A tracer that gathered 192 B at every "
                                      "Runge-Kutta stage would have to move "
                                      "method_bytes_per_stage_rate to match this one"}
    # the ALU roofline's peak is derived from the unit counts; a FMA microbenchmark
    # gives the sustained rate of the same (unpacked) instructions beside it
    fma = valu_fma_rate()
    out["roofline"]["measured_fma_peak"] = fma / 1e12
    out["roofline"]["frac_of_measured"] = achieved / fma
    if other is not None:
        oms = other_flight["ms"] if other_flight else other["ms"]
        out["f64_form"] = {"value": npts / (oms * 1e-3), "ms_per_step": oms, "maps_in_flight": nfl,
                           "one_map_at_a_time": {"value": npts / (other["ms"] * 1e-3),
                                                 "ms_per_step": other["ms"]},
                           "trace_ms": other["trace_ms"]}
    if not args.no_seeds:
        # the same workload drawn with the two other seeds (the value above is seed's)
        seeds = {}
        for sd in [x for x in (0, 1, 2) if x != args.seed][:2]:
            ws_ = synth.config_c2(sd)
            rr = run_gpu(ws_, args.precision, args.tol, args.sub_steps, args.warmup)
            # as the headline: maps in flight, and one at a time beside it
            fl = run_in_flight(ws_, args.precision, args.tol, args.steps, args.warmup, nfl) if nfl > 1 else None
            fms = fl["ms"] if fl else rr["ms"]
            seeds[str(sd)] = {"value": npts / (fms * 1e-3), "ms_per_step": fms, "maps_in_flight": nfl,
                              "one_map_at_a_time": {"value": npts / (rr["ms"] * 1e-3),
                                                    "ms_per_step": rr["ms"]},
                              "trial_steps": rr["stats"][0]}
            del ws_, rr, fl
        out["config"]["other_seeds"] = seeds
    if not args.no_variants and args.precision == "f32x" and other is not None:
        # the variants run one map at a time: their ratios are taken to that form
        uv = {"f32x": seq_value, "f64": npts / (other["ms"] * 1e-3)}
        ws_ = synth.config_c2s(args.seed)
        out["stretched"] = run_variant(
            ws_, "C2 on a stretched grid of the same node counts (x, y clustered at the centre, "
                 "cells 0.67x-1.7x the mean width; z cells growing 1% per cell, 0.5x-1.75x); "
                 "the paper reports 45-80% of its uniform-grid throughput there", args, uv)
        del ws_
        out["method2"] = run_variant(
            w, "C2, Method II (Q, Q_perp and Tw from U, V traced with each line; no "
               "neighbour lines)", args, uv, method=1)
    if not args.no_batch:
        out["batch"] = run_batch(args.seed, args.sub_steps, args.warmup)
    if not args.no_adjoint:
        out["adjoint"] = run_adjoint(args.seed, args.sub_steps, args.warmup)
        out["adjoint_f32x"] = run_adjoint(args.seed, args.sub_steps, args.warmup, "f32x")
    q3d_sample = None
    if not args.no_q3d:
        out["q3d"] = run_q3d(args.seed, args.sub_steps, args.warmup)
        q3d_sample = out["q3d"].pop("_sample")
        # its FP32 pass against the same walks on a record array of its cube's size
        fp = out["q3d"]["f32x"].get("fp32_pass")
        c3 = by_size.get("512x512x256 (C3)")
        if fp and c3:
            fp["gather_frac_of_coherent_walks"] = fp["gathered_GB_per_s"] / c3["coherent"]
            fp["gather_vs_incoherent_walks"] = fp["gathered_GB_per_s"] / c3["incoherent"]
    if args.calib_copy:
        import torch

        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, args.cpu_side)
        orc_map, at = cb.pop("_map"), cb.pop("_at")
        log(f"cpu baseline: {cb}")
        cb.pop("finite_q", None)
        out["cpu_baseline"] = cb
        out["cpu_baseline"]["c1_full_map"] = cpu_c1_rows()
        log(f"oracle on the full C1 map: {out['cpu_baseline']['c1_full_map']}")
        # the accuracy the throughput is stated at
        out["accuracy"] = {args.precision: accuracy(main_run["map"], orc_map, at, w)}
        out["accuracy"][args.precision].update(
            foot_stats(block_ends(w, main_run["params"], at), orc_map, at[2]))
        if other is not None:
            out["accuracy"]["f64"] = accuracy(other["map"], orc_map, at, w)
            out["accuracy"]["f64"].update(foot_stats(block_ends(w, other["params"], at), orc_map, at[2]))
        log(f"accuracy: {out['accuracy']}")
        if q3d_sample is not None:
            out["q3d"]["accuracy"] = q3d_accuracy(*q3d_sample)
            log(f"q3d accuracy: {out['q3d']['accuracy']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
