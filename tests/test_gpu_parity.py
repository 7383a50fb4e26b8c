"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import Plane, cubic_grid, linear_field

from gpu_util import TOL_TW, compare_maps, compare_points, to_np

pytestmark = pytest.mark.gpu

F32X, F64 = 0, 1
ORC_TOL = {"tol": 1e-10}


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


def _dev(B):
    import torch

    return torch.from_numpy(np.ascontiguousarray(B)).cuda()


def _run_q2d(fq, B, grid, plane, prec, **kw):
    import torch

    p = fq.Params(precision=prec, **kw)
    r = fq.q2d(_dev(B), grid, plane, p, want_lines=True)
    torch.cuda.synchronize()
    return r


@pytest.fixture(scope="module")
def c1():
    w = synth.config_c1(0)
    o = oracle.q2d(w.field, w.grid, w.plane, ORC_TOL)
    return w, o


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_c1_full_map_parity(fq, c1, prec):
    """The 128x128 Q/Tw map of the 4-charge 64^3 cube, every point."""
    w, o = c1
    _say(f"c1 full map, precision {prec}")
    g = _run_q2d(fq, w.field, w.grid, w.plane, prec)
    st = compare_maps(g, o, f"c1-{prec}")
    print(st)
    assert st["excluded_frac"] < 0.02


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_ragged_seed_grid_and_fp32_field(fq, prec):
    """Seed grids that are not multiples of the 8x8 queue tile, on an FP32 cube."""
    rng = np.random.default_rng(5)
    g = cubic_grid(40, 36, 30)
    pos, q = synth.draw_charges(rng, 6)
    B = synth.charges_field(g, pos, q, dtype=np.float32)
    ux, uy, _ = g.upper
    pl = Plane((0.013, 0.021, 0.0), (1, 0, 0), (0, 1, 0), 61, 45, (ux - 0.03) / 61, (uy - 0.05) / 45)
    _say(f"ragged 61x45 seeds on 40x36x30 fp32, precision {prec}")
    o = oracle.q2d(B, g, pl, ORC_TOL)
    r = _run_q2d(fq, B, g, pl, prec)
    st = compare_maps(r, o, "ragged")
    print(st)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_closed_form_fields(fq, prec):
    """Sheared (Q = 2 + s^2 L^2, Tw closed form), hyperbolic (Q = 2 cosh 2kL) and
    twisted (Tw = qL / (2 pi sqrt(1 + q^2 rho^2))) fields on the GPU."""
    g = cubic_grid(17, 17, 17)
    s, y0 = 0.5, 0.5
    B = linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1])
    pl = Plane((0.41, 0.25, 0.0), (1, 0, 0), (0, 1, 0), 9, 9, 0.02, 0.02)
    _say(f"shear field, precision {prec}")
    r = _run_q2d(fq, B, g, pl, prec)
    q = to_np(r["q"])
    assert np.allclose(q[1:-1, 1:-1], 2 + s * s, rtol=1e-5)
    y1 = pl.points()[:, 1].reshape(9, 9)
    tw = -s / (4 * np.pi * np.sqrt(1 + s * s * (y1 - y0) ** 2))
    assert np.allclose(to_np(r["tw"]), tw, atol=TOL_TW)

    kL = 4.0
    B = linear_field(g, [[kL, 0, 0], [0, -kL, 0], [0, 0, 0]], [-kL * 0.5, kL * 0.5, 1])
    d = 1e-4
    pl = Plane((0.5 + 0.1 * math.exp(-kL) - d, 0.6 - d, 0.0), (1, 0, 0), (0, 1, 0), 3, 3, d, d)
    _say(f"hyperbolic field, precision {prec}")
    r = _run_q2d(fq, B, g, pl, prec)
    qexp = 2 * math.cosh(2 * kL)
    qg = to_np(r["q"])[1, 1]
    assert abs(math.log10(qg) / math.log10(qexp) - 1) < 1e-4, (qg, qexp)

    qt = 3 * math.pi
    B = linear_field(g, [[0, -qt, 0], [qt, 0, 0], [0, 0, 0]], [qt * 0.5, -qt * 0.5, 1.0])
    pl = Plane((0.53, 0.48, 0.0), (1, 0, 0), (0, 1, 0), 4, 4, 0.01, 0.01)
    _say(f"twisted field, precision {prec}")
    r = _run_q2d(fq, B, g, pl, prec)
    pts = pl.points()
    rho = np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5)
    tw = qt / (2 * np.pi * np.sqrt(1 + qt * qt * rho * rho))
    assert np.allclose(to_np(r["tw"]).ravel(), tw, atol=TOL_TW)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_end_on_box_face_just_before_a_cell_face(fq, prec):
    """B = (1, 0, -(x - x0)): from the apex (x0, y, m^2/2) the lines are parabolas that
    leave through the bottom face at x0 +- m with slope m (Eq. rb). With the forward
    exit a distance eps before an x face, a step aimed at the x face ends just below
    the box; clamping that end onto z = 0 would move it by up to eps. The ends must
    match the closed form. Slopes of 0.08 and 0.2 keep the ends out of the FP64
    re-trace, so the F32X form checks the FP32 pass itself."""
    import torch

    g = cubic_grid(17, 17, 17)
    _say(f"box-face ends near x faces, precision {prec}")
    for xf in (0.4375, 0.5625):
        for eps in (1e-6, 3e-6, 6e-6, 2e-5):
            for m in (0.08, 0.2):
                x0 = xf - eps - m
                B = linear_field(g, [[0, 0, 0], [0, 0, 0], [-1, 0, 0]], [1.0, 0.0, x0])
                seeds = np.array([[x0, 0.53, m * m / 2]])
                r = fq.trace(_dev(B), g, torch.from_numpy(seeds).cuda(), normal=(1.0, 0.0, 0.0),
                             params=fq.Params(precision=prec))
                torch.cuda.synchronize()
                assert int(to_np(r["status"])[0]) == 0
                assert int(to_np(r["face_f"])[0]) == 4 and int(to_np(r["face_b"])[0]) == 4
                for key, xe in (("end_f", x0 + m), ("end_b", x0 - m)):
                    e = to_np(r[key])[0]
                    assert np.max(np.abs(e - [xe, 0.53, 0.0])) < 1e-7, (xf, eps, m, key, e)


def test_status_paths(fq):
    """Seeds outside the box, a NaN in the field, a null region and the step budget
    are reported per line, as in the oracle."""
    import torch

    g = cubic_grid(9, 9, 9)
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    seeds = np.array([[1.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5, 0.5, 0.1]])
    _say("status paths: outside seed")
    r = fq.trace(_dev(B), g, torch.from_numpy(seeds).cuda())
    torch.cuda.synchronize()
    st = to_np(r["status"]).astype(np.uint16)
    assert st[0] & fq.ST_OUTSIDE and st[1] == 0 and st[2] == 0
    assert math.isnan(to_np(r["tw"])[0])
    Bn = B.copy()
    Bn[2, 6, 4, 4] = np.nan
    _say("status paths: NaN in field")
    r = fq.trace(_dev(Bn), g, torch.from_numpy(seeds[2:]).cuda())
    torch.cuda.synchronize()
    assert to_np(r["status"])[0] & fq.ST_NONFINITE
    Bz = B.copy()
    Bz[:, 5:, :, :] = 0.0
    _say("status paths: null region")
    r = fq.trace(_dev(Bz), g, torch.from_numpy(seeds[2:]).cuda())
    torch.cuda.synchronize()
    assert to_np(r["status"])[0] & fq.ST_NULLB
    _say("status paths: step budget")
    r = fq.trace(_dev(B), g, torch.from_numpy(seeds[2:]).cuda(), params=fq.Params(max_steps=1))
    torch.cuda.synchronize()
    assert to_np(r["status"])[0] & fq.ST_MAXSTEPS


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_trace_list_matches_oracle(fq, prec):
    """fastqsl_trace on arbitrary seeds (interior and on faces) against the oracle."""
    import torch

    w = synth.config_c1(1)
    rng = np.random.default_rng(11)
    seeds = np.concatenate([rng.uniform(0.02, 0.98, (300, 3)),
                            np.c_[rng.uniform(0.05, 0.95, (100, 2)), np.zeros(100)]])
    _say(f"trace list of 400 seeds, precision {prec}")
    r = fq.trace(_dev(w.field), w.grid, torch.from_numpy(seeds).cuda(),
                 params=fq.Params(precision=prec))
    torch.cuda.synchronize()
    o = oracle.trace(w.field, w.grid, seeds, opts=ORC_TOL)
    sg = to_np(r["status"]).astype(np.uint16)
    ok = ((sg | o["status"]) & (oracle.FATAL | oracle.ORC_EDGE)) == 0
    assert ok.mean() > 0.9
    for k in ("end_b", "end_f"):
        d = np.max(np.abs(to_np(r[k]) - o[k]), axis=1)
        assert d[ok].max() < 1e-6, (k, d[ok].max())
    assert np.array_equal(to_np(r["face_b"])[ok], o["face_b"][ok])
    assert np.abs(to_np(r["tw"])[ok] - o["tw"][ok]).max() < TOL_TW
    assert np.allclose(to_np(r["length"])[ok], o["len"][ok], rtol=1e-6, atol=1e-7)
    assert np.allclose(to_np(r["bn0"])[ok], o["bn0"][ok], rtol=1e-12, atol=1e-12)
    # B_n at an end follows the end point (which agrees to ~1e-7)
    assert np.allclose(to_np(r["bn_f"])[ok], o["bn_f"][ok], rtol=1e-5, atol=1e-6)


def test_batched_equals_single(fq):
    """Two cubes of different sizes in one persistent launch give bit-identical maps
    to the same jobs launched alone."""
    import torch

    jobs = synth.config_c4(3, njobs=2, edge=(40, 72), sides=(64, 96), ncharge=(4, 6))
    _say("batched 2 jobs")
    dev = [(_dev(j.field), j.grid, j.plane) for j in jobs]
    rb = fq.q2d_batch(dev, fq.Params(), want_lines=False)
    torch.cuda.synchronize()
    for (B, g, pl), r in zip(dev, rb):
        r1 = fq.q2d(B, g, pl, fq.Params())
        torch.cuda.synchronize()
        a, b = to_np(r["q"]), to_np(r1["q"])
        assert np.array_equal(np.isnan(a), np.isnan(b))
        assert np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])
        assert np.array_equal(to_np(r["tw"]), to_np(r1["tw"]), equal_nan=True)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_batch_with_a_job_smaller_than_a_refill(fq, prec):
    """A job of 12 half lines (fewer than the idle lanes a wave waits for before it
    refills, in FP32; about that many in FP64) next to two larger cubes in one
    launch: every job's map equals the job launched alone, bit for bit."""
    import torch

    jobs = synth.config_c4(5, njobs=2, edge=(40, 72), sides=(64, 96), ncharge=(4, 6))
    dev = [(_dev(j.field), j.grid, j.plane) for j in jobs]
    g = jobs[0].grid
    tiny = Plane((0.4, 0.45, 0.0), (1, 0, 0), (0, 1, 0), 2, 3, 0.01, 0.01)
    dev.append((dev[0][0], g, tiny))
    _say(f"batch with a 2x3 job, precision {prec}")
    rb = fq.q2d_batch(dev, fq.Params(precision=prec), want_lines=False)
    torch.cuda.synchronize()
    assert to_np(rb[2]["q"]).shape == (3, 2)
    for (B, gg, pl), r in zip(dev, rb):
        r1 = fq.q2d(B, gg, pl, fq.Params(precision=prec))
        torch.cuda.synchronize()
        for k in ("q", "tw", "length"):
            assert np.array_equal(to_np(r[k]), to_np(r1[k]), equal_nan=True), k
        assert np.array_equal(to_np(r["status"]), to_np(r1["status"]))
    assert np.isfinite(to_np(rb[2]["length"])).all()


def test_deterministic(fq, c1):
    w, _ = c1
    _say("determinism: two runs")
    a = _run_q2d(fq, w.field, w.grid, w.plane, F32X)
    b = _run_q2d(fq, w.field, w.grid, w.plane, F32X)
    assert np.array_equal(to_np(a["q"]), to_np(b["q"]), equal_nan=True)
    assert np.array_equal(to_np(a["tw"]), to_np(b["tw"]), equal_nan=True)


def test_degenerate_inputs(fq):
    """A 1x1 map (no neighbours: MIXEDFACE), a 2x2x2 cube, an empty trace."""
    import torch

    g = cubic_grid(2, 2, 2)
    B = linear_field(g, np.zeros((3, 3)), [0.1, 0.0, 1.0])
    pl = Plane((0.5, 0.5, 0.0), (1, 0, 0), (0, 1, 0), 1, 1, 0.1, 0.1)
    _say("1x1 map on a 2x2x2 cube")
    r = _run_q2d(fq, B, g, pl, F32X)
    assert to_np(r["status"])[0, 0] & fq.ST_MIXEDFACE
    assert abs(to_np(r["length"])[0, 0] - math.sqrt(1 + 0.01)) < 1e-6
    pl = Plane((0.3, 0.3, 0.0), (1, 0, 0), (0, 1, 0), 3, 3, 0.1, 0.1)
    r = _run_q2d(fq, B, g, pl, F32X)
    assert abs(to_np(r["q"])[1, 1] - 2.0) < 1e-5
    _say("empty trace")
    out = fq.trace(_dev(B), g, torch.zeros((0, 3), dtype=torch.float64).cuda())
    assert out["status"].numel() == 0


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_q3d_small_matches_oracle(fq, prec):
    """3-D maps (one line per voxel, rotated S0 where |Bz/B| < 0.05) on a small cube."""
    import torch

    rng = np.random.default_rng(2)
    g = cubic_grid(33, 33, 25)
    pos, q = synth.draw_charges(rng, 6)
    B = synth.charges_field(g, pos, q)
    ux, uy, uz = g.upper
    vx = synth.Voxels((ux / 32, uy / 32, uz / 20), (ux / 16, uy / 16, uz / 10), (15, 15, 9))
    _say(f"q3d 15x15x9 voxels, precision {prec}")
    o = oracle.q3d(B, g, vx, ORC_TOL)
    r = fq.q3d(_dev(B), g, vx, fq.Params(precision=prec), want_lines=True)
    torch.cuda.synchronize()
    rot = (o["status"] & oracle.ORC_ROTATED) != 0
    st = compare_maps(r, o, "q3d")
    print(st, "rotated points:", int(rot.sum()))


def _sample(n_total, nu, nv, k, seed):
    """k random map points plus the four corners and some edge points."""
    rng = np.random.default_rng(seed)
    pts = rng.choice(n_total, k, replace=False)
    edge = [0, nu - 1, nu * (nv - 1), nu * nv - 1, nu // 2, nu * (nv // 2)]
    return np.unique(np.concatenate([pts, edge]))


@pytest.fixture(scope="module")
def c2():
    return synth.config_c2(0)


C2_BLOCK = 512


@pytest.fixture(scope="module")
def c2_block(c2):
    """The oracle on the central 512 x 512 block of the C2 seed grid (every line of
    the block traced in FP64 and assembled with its neighbours in the block)."""
    w = c2
    pl = w.plane
    i0 = (pl.nu - C2_BLOCK) // 2
    j0 = (pl.nv - C2_BLOCK) // 2
    o = np.asarray(pl.origin) + i0 * pl.du * np.asarray(pl.u) + j0 * pl.dv * np.asarray(pl.v)
    sub = Plane(tuple(o), pl.u, pl.v, C2_BLOCK, C2_BLOCK, pl.du, pl.dv)
    _say("c2 oracle block 512x512 (CPU)")
    return (i0, j0), oracle.q2d(w.field, w.grid, sub, ORC_TOL)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_c2_full_size_block_parity(fq, c2, c2_block, prec):
    """The 1024x1024 map of the 256x256x128 FP32 cube (6 charges + twisted tube), in
    the launch configuration the bench times, against the oracle on every point of
    the central 512 x 512 block whose stencil lies inside the block (510 x 510
    points, footpoints included), with the parity mask and tolerances of every
    other map test: no exception for seeds near polarity inversion lines."""
    import torch

    w = c2
    _say(f"c2 1024x1024 full map, precision {prec}")
    r = fq.q2d(_dev(w.field), w.grid, w.plane, fq.Params(precision=prec), want_lines=True)
    torch.cuda.synchronize()
    (i0, j0), o = c2_block
    n = C2_BLOCK
    sl = (slice(j0 + 1, j0 + n - 1), slice(i0 + 1, i0 + n - 1))

    def gblock(t, last=None):
        a = to_np(t)
        if last is None:
            return a.reshape(1024, 1024)[sl].ravel()
        return a.reshape(1024, 1024, last)[sl].reshape(-1, last)

    def oblock(a, last=None):
        a = np.asarray(a)
        if last is None:
            return a.reshape(n, n)[1:-1, 1:-1].ravel()
        return a.reshape(n, n, last)[1:-1, 1:-1].reshape(-1, last)

    g = {"q": gblock(r["q"]), "tw": gblock(r["tw"]), "status": gblock(r["status"]),
         "lines": {k: gblock(r["lines"][k], 3 if k.startswith("end") else None)
                   for k in ("end_b", "end_f", "face_b", "face_f")}}
    ob = {"q": oblock(o["q"]), "tw": oblock(o["tw"]), "status": oblock(o["status"]),
          "lines": {k: oblock(o["lines"][k], 3 if k.startswith("end") else None)
                    for k in ("end_b", "end_f", "face_b", "face_f")}}
    st = compare_maps(g, ob, f"c2-block-{prec}", raw=True)
    print(st)
    assert st["excluded_frac"] < 0.05
    # properties that hold everywhere: no failed lines, Tw finite on every line
    sg = to_np(r["status"]).astype(np.uint16)
    assert not (sg & fq.ST_FATAL).any()
    assert np.isfinite(to_np(r["tw"])).all()


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_c2_high_q_points_parity(fq, prec):
    """The same workload drawn with seed 1, whose map has a wide high-Q region, where
    the map stretches each line's rounding by about sqrt(Q). Against the oracle: the
    200 lines whose ends move most between this form and an FP64 map at a 1000x
    tighter tolerance (the GPU map only picks the points; the oracle gives the
    values), the 100 largest-Q points and 100 random ones, footpoints included. In
    the F32X form, lines whose point has Q > 300 are re-traced in FP64."""
    import torch

    w = synth.config_c2(1)
    B = _dev(w.field)
    _say(f"c2 seed 1 high-Q points, precision {prec}")
    r = fq.q2d(B, w.grid, w.plane, fq.Params(precision=prec), want_lines=True)
    ref = fq.q2d(B, w.grid, w.plane, fq.Params(precision=F64, tol_perp=1e-9), want_lines=True)
    torch.cuda.synchronize()
    d = np.zeros(1024 * 1024)
    for k in ("end_b", "end_f"):
        d = np.maximum(d, np.abs(to_np(r["lines"][k]) - to_np(ref["lines"][k])).max(axis=1))
    d = np.where(np.isfinite(d), d, 0.0)
    q = to_np(r["q"]).ravel()
    qs = np.where(np.isfinite(q) & (q < 1e8), q, 0.0)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([np.argsort(-d)[:200], np.argsort(-qs)[:100],
                                    rng.choice(q.size, 100, replace=False)]))
    o = oracle.q2d_points(w.field, w.grid, w.plane, idx, ORC_TOL)
    st = compare_points(r, idx, o, f"c2-seed1-highq-{prec}")
    print(st, "largest end shift:", float(d.max()), "largest Q:", float(qs.max()))
    assert qs.max() > 1e4


@pytest.fixture(scope="module")
def c3():
    return synth.config_c3(0)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_c3_full_size_sampled_parity(fq, c3, prec):
    """3-D Q and Tw on the 256x256x128 voxel centres of the 512x512x256 FP32 cube
    (10 charges + two tubes), including rotated-S0 voxels, against the oracle at
    sampled voxels: 300 random ones, 60 random rotated ones and the 40 rotated ones
    with the largest Q below 1e8 (where the F32X form re-traces all four of a
    rotated voxel's lines in FP64)."""
    import torch

    w = c3
    vx = w.voxels
    _say(f"c3 q3d 256x256x128 voxels, precision {prec}")
    r = fq.q3d(_dev(w.field), w.grid, vx, fq.Params(precision=prec), want_lines=True)
    torch.cuda.synchronize()
    n = int(np.prod(vx.n))
    st_all = to_np(r["status"]).astype(np.uint16).ravel()
    rot = np.flatnonzero(st_all & fq.ST_ROTATED)
    rng = np.random.default_rng(23)
    q_all = to_np(r["q"]).ravel()
    qr = q_all[rot]
    ok = np.isfinite(qr) & (qr < 1e8)
    top = rot[ok][np.argsort(qr[ok])[-40:]]
    idx = np.unique(np.concatenate([rng.choice(n, 300, replace=False),
                                    rng.choice(rot, min(60, rot.size), replace=False), top]))
    print("largest Q among the rotated voxels compared:", float(q_all[top].max()))
    o = oracle.q3d_points(w.field, w.grid, vx, idx, ORC_TOL)
    st = compare_points(r, idx, o, f"c3-{prec}")
    print(st, "rotated voxels:", rot.size)
    assert rot.size > 0
    assert not (st_all & fq.ST_FATAL).any()


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_batch_with_interior_planes_equals_single(fq, prec):
    """Interior seed planes (rotated S0 where |Bn0/B| < 0.05, four extra lines each)
    and a box-face plane in one persistent launch: the rotated-S0 jobs' queue ranges
    are sized on the device, one after another, and every map is bit-identical to
    the same job launched alone."""
    import torch

    w = synth.config_c1(0)
    B = _dev(w.field)
    planes = [Plane((0.11, 0.13, 0.37), (1, 0, 0), (0, 1, 0), 40, 36, 0.02, 0.02),
              Plane((0.2, 0.31, 0.21), (1, 0, 0), (0, 0.6, 0.8), 30, 28, 0.02, 0.02),
              Plane((0.05, 0.05, 0.0), (1, 0, 0), (0, 1, 0), 48, 40, 0.018, 0.02)]
    _say(f"batch of two interior planes and a face plane, precision {prec}")
    p = fq.Params(precision=prec)
    rb = fq.q2d_batch([(B, w.grid, pl) for pl in planes], p, want_lines=False)
    torch.cuda.synchronize()
    nrot = 0
    for pl, r in zip(planes, rb):
        r1 = fq.q2d(B, w.grid, pl, p)
        torch.cuda.synchronize()
        a, b = to_np(r["q"]), to_np(r1["q"])
        assert np.array_equal(np.isnan(a), np.isnan(b))
        assert np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])
        assert np.array_equal(to_np(r["tw"]), to_np(r1["tw"]), equal_nan=True)
        assert np.array_equal(to_np(r["status"]), to_np(r1["status"]))
        nrot += int(((to_np(r["status"]).astype(np.uint16) & fq.ST_ROTATED) != 0).sum())
    assert nrot > 0
