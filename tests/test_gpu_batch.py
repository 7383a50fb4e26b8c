"""Batching, HIP-graph capture and the autotuner, through the C-ABI.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import sys

import numpy as np
import pytest

import oracle
import synth
from synth import cubic_grid, plane_z0

from gpu_util import compare_maps, compare_points, to_np

pytestmark = pytest.mark.gpu

F32X, F64 = 0, 1
ORC_TOL = {"tol": 1e-10}
KEYS = ("q", "tw", "length", "status")
LINE_KEYS = ("end_b", "end_f", "face_b", "face_f", "bn_b", "bn_f", "bn0", "tw", "length", "status")


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fq():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2208_12569_amd as m

    m._lib.load()
    return m


def _same(a: dict, b: dict, label: str):
    """Bitwise equality of two maps (NaN == NaN)."""
    for k in KEYS:
        x, y = to_np(a[k]), to_np(b[k])
        assert np.array_equal(x, y, equal_nan=True), (label, k)
    if "lines" in a and "lines" in b:
        for k in LINE_KEYS:
            x, y = to_np(a["lines"][k]), to_np(b["lines"][k])
            assert np.array_equal(x, y, equal_nan=True), (label, "lines", k)


def _small_batch(seed: int):
    """Three uneven cubes (FP32 and FP64 fields) with ragged seed grids."""
    rng = np.random.default_rng(seed)
    out = []
    for E, side, dt in ((48, 72, np.float32), (33, 40, np.float64), (64, 96, np.float32)):
        g = cubic_grid(E, E, E)
        pos, q = synth.draw_charges(rng, 5)
        out.append((synth.charges_field(g, pos, q, dtype=dt), g, plane_z0(side)))
    return out


def _dev(jobs):
    import torch

    return [(torch.from_numpy(np.ascontiguousarray(B)).cuda(), g, pl) for B, g, pl in jobs]


@pytest.mark.parametrize("prec,in_flight", [(F32X, False), (F64, False), (F32X, True)],
                         ids=["f32x", "f64", "f32x-in-flight"])
def test_graph_replays_match_eager(fq, prec, in_flight):
    """A captured batch replayed three times, with the fields rewritten in place and
    eager work between replays, equals eager calls bit for bit every time (also with
    in_flight, whose FP64 pass takes its list through a counting sort)."""
    import torch

    from paper_2208_12569_amd.graph import Q2DGraph

    _say(f"graph replay, 3-cube batch, precision {prec}, in_flight {in_flight}")
    A = _dev(_small_batch(1))
    Bj = _dev(_small_batch(2))
    p = fq.Params(precision=prec)
    ref_a = fq.q2d_batch(A, p, want_lines=True)
    ref_b = fq.q2d_batch(Bj, p, want_lines=True)
    torch.cuda.synchronize()
    keep = [B.clone() for B, _, _ in A]
    g = Q2DGraph(A, fq.Params(precision=prec, in_flight=in_flight), want_lines=True)
    for it, (src, ref) in enumerate(((None, ref_a), (Bj, ref_b), (keep, ref_a))):
        if src is not None:
            for (dst, _, _), s in zip(A, src):
                dst.copy_(s[0] if isinstance(s, tuple) else s)
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        outs = g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for j, (o, r) in enumerate(zip(outs, ref)):
            _same(o, r, f"replay {it} job {j}")


def test_launch_shapes_do_not_change_results(fq):
    """Block size and grid size only change scheduling: maps are identical, and the
    tuner returns one of the candidates."""
    import torch

    from paper_2208_12569_amd.tune import tune_launch

    _say("launch shapes, one 64^3 job")
    jobs = _dev(_small_batch(3)[2:])
    ref = fq.q2d_batch(jobs, fq.Params(), want_lines=True)
    for block, waves in ((64, 0), (128, 4), (192, 12), (256, 1)):
        r = fq.q2d_batch(jobs, fq.Params(block=block, waves_per_cu=waves), want_lines=True)
        torch.cuda.synchronize()
        _same(r[0], ref[0], f"block {block} waves {waves}")
    p, table = tune_launch(jobs, fq.Params(), blocks=(64, 256), waves=(0, 4), reps=1)
    assert (p.block, p.waves_per_cu) in table and len(table) == 4
    assert all(v > 0 for v in table.values())


def test_tuned_tolerance_meets_the_bar(fq):
    """The tolerance the tuner accepts (checked only against the all-FP64 form) also
    keeps the C1 map within the parity bar against the oracle."""
    import torch

    from paper_2208_12569_amd.tune import tune_tol

    w = synth.config_c1(0)
    _say("tolerance tuner on c1")
    jobs = _dev([(w.field, w.grid, w.plane)])
    p, report = tune_tol(jobs, fq.Params(), tols=(1e-4, 1e-5, 1e-6), reps=1)
    print(p.tol_perp, report)
    assert report[1e-6]["ok"]
    assert p.tol_perp in report and report[p.tol_perp]["ok"]
    r = fq.q2d(jobs[0][0], w.grid, w.plane, p, want_lines=True)
    torch.cuda.synchronize()
    o = oracle.q2d(w.field, w.grid, w.plane, ORC_TOL)
    st = compare_maps(r, o, f"c1 tuned tol {p.tol_perp}")
    print(st)


@pytest.fixture(scope="module")
def c4():
    from synth.torch_fields import config_c4_torch

    _say("generating the 16-cube batch on the GPU")
    return config_c4_torch(0)


def test_c4_batch_in_graph(fq, c4):
    """The 16 uneven cubes (edges 64-384, seed grids 128^2-1024^2) in one persistent
    launch captured in a HIP graph, with tuned launch parameters: every job equals
    the same job run alone, and sampled points match the oracle."""
    import torch

    from paper_2208_12569_amd.graph import Q2DGraph
    from paper_2208_12569_amd.tune import autotune

    jobs = [(w.field, w.grid, w.plane) for w in c4]
    _say("c4 batch: tuning")
    p = autotune(jobs, fq.Params(), reps=1)
    _say(f"c4 batch: graph with block {p.block}, waves/CU {p.waves_per_cu}")
    g = Q2DGraph(jobs, p, want_lines=True)
    outs = g.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(41)
    for j, (w, o) in enumerate(zip(c4, outs)):
        _say(f"c4 job {j} ({w.name}) alone")
        alone = fq.q2d(w.field, w.grid, w.plane, p, want_lines=True)
        torch.cuda.synchronize()
        _same(o, alone, f"c4 job {j}")
        st = to_np(o["status"]).astype(np.uint16)
        assert not (st & fq.ST_FATAL).any(), w.name
        n = w.plane.nu * w.plane.nv
        idx = np.unique(rng.choice(n, 24, replace=False))
        Bh = w.field.cpu().numpy()
        ores = oracle.q2d_points(Bh, w.grid, w.plane, idx, ORC_TOL)
        s = compare_points(o, idx, ores, f"c4 {w.name}")
        print(w.name, s)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_maps_in_flight_on_several_streams(fq, prec):
    """Maps computed four at a time on four streams of default priority, each with
    its own workspace (one map's FP64 pass overlapping the others' FP32 passes, run in
    its three-waves-per-SIMD form: in_flight), equal the same maps computed one at a
    time, bit for bit: a face plane, an interior plane with rotated-S0 points and a
    3-D map, three rounds over the streams."""
    import dataclasses

    import torch

    g = cubic_grid(48, 48, 40)
    pos, q = synth.draw_charges(np.random.default_rng(17), 6)
    B = torch.from_numpy(synth.charges_field(g, pos, q, dtype=np.float32)).cuda()
    p = fq.Params(precision=prec)
    face = plane_z0(56)
    mid = synth.Plane((0.1, 0.1, 0.37), (1, 0, 0), (0, 1, 0), 40, 36, 0.02, 0.022)
    vx = synth.Voxels((0.1, 0.1, 0.1), (0.05, 0.05, 0.1), (16, 16, 5))
    pf = dataclasses.replace(p, in_flight=True)
    calls = [lambda s, ws, q: fq.q2d(B, g, face, q, want_lines=True, stream=s, ws=ws),
             lambda s, ws, q: fq.q2d(B, g, mid, q, want_lines=True, stream=s, ws=ws),
             lambda s, ws, q: fq.q3d(B, g, vx, q, want_lines=True, stream=s, ws=ws)]
    _say(f"maps one at a time, precision {prec}")
    ref = [c(None, None, p) for c in calls]
    torch.cuda.synchronize()
    assert bool(((ref[1]["status"].to(torch.int32) & fq.ST_ROTATED) != 0).any())
    streams = [torch.cuda.Stream() for _ in range(4)]
    wss = {}
    outs = []
    _say(f"maps four in flight, precision {prec}")
    for rnd in range(3):
        for k, c in enumerate(calls):
            i = rnd * len(calls) + k
            s = streams[i % 4]
            with torch.cuda.stream(s):
                r = c(s, wss.get((i % 4, k)), pf)
            wss[(i % 4, k)] = r["_ws"]
            outs.append((k, r))
    torch.cuda.synchronize()
    for n, (k, r) in enumerate(outs):
        _same(r, ref[k], f"in flight {n} (call {k})")


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_q2d_many_equals_one_at_a_time(fq, prec):
    """q2d_many (maps three in flight on three streams) over seven jobs of uneven
    cubes and seed grids, FP32 and FP64 fields, an interior plane among them: each map
    equals its own q2d call bit for bit, and is ready on the caller's stream."""
    import torch

    jobs = _dev(_small_batch(5)) + _dev(_small_batch(6))
    B, g, _ = jobs[0]
    jobs.append((B, g, synth.Plane((0.1, 0.1, 0.41), (1, 0, 0), (0, 1, 0), 30, 26, 0.025, 0.03)))
    p = fq.Params(precision=prec)
    _say(f"q2d_many over {len(jobs)} jobs, precision {prec}")
    many = fq.q2d_many(jobs, p, want_lines=True)
    for j, ((B, g, pl), r) in enumerate(zip(jobs, many)):
        ref = fq.q2d(B, g, pl, p, want_lines=True)
        torch.cuda.synchronize()
        _same(r, ref, f"q2d_many job {j}")
