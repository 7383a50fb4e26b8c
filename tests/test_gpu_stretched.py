"""Stretched rectilinear grids (Section 2.2: nodes x_i, y_j, z_k, the cell of a
point by bisection; Section 2.3: step and tol scaled per cell) on the GPU, through
the C-ABI, in both forms: closed forms of linear fields, full-map parity with the
oracle on the stretched 4-charge cube, explicit uniform nodes against the uniform
grid, batches, 3-D maps, and malformed node coordinates.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import Plane, linear_field

from gpu_util import TOL_LOGQ, TOL_TW, compare_maps, to_np

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


def _q2d(fq, B, grid, plane, prec, **kw):
    import torch

    r = fq.q2d(_dev(B), grid, plane, fq.Params(precision=prec, **kw), want_lines=True)
    torch.cuda.synchronize()
    return r


def _random_stretched(nx, ny, nz, seed, hi=(1.0, 1.0, 1.0)):
    """Cell widths drawn in [0.3, 1.7] times the mean: neighbouring cells differ by up
    to a factor of five."""
    rng = np.random.default_rng(seed)
    ax = []
    for n, b in zip((nx, ny, nz), hi):
        w = rng.uniform(0.3, 1.7, n - 1)
        x = np.concatenate([[0.0], np.cumsum(w)]) * (b / w.sum())
        x[-1] = b
        ax.append(x)
    return synth.stretched_grid(*ax)


def _logq_ok(got, exp):
    le = np.log10(np.asarray(exp, float))
    return np.abs(np.log10(np.asarray(got, float)) - le) / np.maximum(np.abs(le), math.log10(2)) <= TOL_LOGQ


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_stretched_closed_forms(fq, prec):
    """Linear fields are their own trilinear interpolants on any rectilinear grid:
    the identity map (Q = 2, length Lz), the sheared field (Q = 2 + s^2, Tw closed
    form, x2 = x1 + s (y1 - y0)), the hyperbolic field (Q = 2 cosh 2kL) and the
    twisted field (Tw = qL / (2 pi sqrt(1 + q^2 rho^2))) on a grid whose
    neighbouring cells differ up to five times in width."""
    g = _random_stretched(17, 15, 19, seed=3)
    _say(f"stretched identity map, precision {prec}")
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    pl = Plane((0.05, 0.07, 0.0), (1, 0, 0), (0, 1, 0), 9, 7, 0.1, 0.13)
    r = _q2d(fq, B, g, pl, prec)
    assert np.all((to_np(r["status"]) & fq.ST_FATAL) == 0)
    assert np.allclose(to_np(r["q"]), 2.0, rtol=1e-6)
    assert np.allclose(to_np(r["length"]), 1.0, atol=1e-6)
    assert np.allclose(to_np(r["lines"]["end_f"])[:, :2], pl.points()[:, :2], atol=1e-6)
    s, y0 = 0.5, 0.5
    _say(f"stretched shear, precision {prec}")
    B = linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1])
    pl = Plane((0.41, 0.25, 0.0), (1, 0, 0), (0, 1, 0), 9, 9, 0.02, 0.02)
    r = _q2d(fq, B, g, pl, prec)
    assert _logq_ok(to_np(r["q"])[1:-1, 1:-1], 2 + s * s).all()
    y1 = pl.points()[:, 1]
    assert np.allclose(to_np(r["tw"]).ravel(), -s / (4 * np.pi * np.sqrt(1 + s * s * (y1 - y0) ** 2)),
                       atol=TOL_TW)
    assert np.allclose(to_np(r["lines"]["end_f"])[:, 0], pl.points()[:, 0] + s * (y1 - y0), atol=1e-6)
    kL = 3.0
    _say(f"stretched hyperbolic kL {kL}, precision {prec}")
    B = linear_field(g, [[kL, 0, 0], [0, -kL, 0], [0, 0, 0]], [-kL * 0.5, kL * 0.5, 1])
    d = 1e-4
    pl = Plane((0.5 + 0.1 * math.exp(-kL) - d, 0.6 - d, 0.0), (1, 0, 0), (0, 1, 0), 3, 3, d, d)
    r = _q2d(fq, B, g, pl, prec)
    assert _logq_ok(to_np(r["q"])[1, 1], 2 * math.cosh(2 * kL))
    qt = 2 * math.pi
    _say(f"stretched twisted field, precision {prec}")
    B = linear_field(g, [[0, -qt, 0], [qt, 0, 0], [0, 0, 0]], [qt * 0.5, -qt * 0.5, 1.0])
    pl = Plane((0.53, 0.48, 0.0), (1, 0, 0), (0, 1, 0), 4, 4, 0.01, 0.01)
    r = _q2d(fq, B, g, pl, prec)
    rho = np.hypot(pl.points()[:, 0] - 0.5, pl.points()[:, 1] - 0.5)
    assert np.allclose(to_np(r["tw"]).ravel(), qt / (2 * np.pi * np.sqrt(1 + qt * qt * rho * rho)),
                       atol=TOL_TW)


@pytest.fixture(scope="module")
def c1s():
    w = synth.config_c1s(0)
    return w, oracle.q2d(w.field, w.grid, w.plane, ORC_TOL)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_c1s_full_map_parity(fq, c1s, prec):
    """The 128 x 128 map of the 4-charge cube on a stretched 64^3 grid (x, y
    clustered at the centre, z cells growing 3% per cell) against the oracle on the
    same grid, every point: Q, Tw, footpoints and statuses."""
    w, o = c1s
    _say(f"c1s full map, precision {prec}")
    g = _q2d(fq, w.field, w.grid, w.plane, prec)
    st = compare_maps(g, o, f"c1s-{prec}")
    print(st)
    assert st["excluded_frac"] < 0.02


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_explicit_uniform_nodes_equal_uniform_grid(fq, prec):
    """Node coordinates that are uniform, given explicitly, take the stretched code
    path (bisection, per-cell scales, multi-job kernel) and give the uniform grid's
    map to within the tracing tolerance."""
    w = synth.config_c1(0)
    gs = synth.stretched_grid(*w.grid.axes())
    _say(f"explicit uniform nodes, precision {prec}")
    ru = _q2d(fq, w.field, w.grid, w.plane, prec)
    rs = _q2d(fq, w.field, gs, w.plane, prec)
    qu, qs = to_np(ru["q"]).ravel(), to_np(rs["q"]).ravel()
    su, ss = to_np(ru["status"]).ravel(), to_np(rs["status"]).ravel()
    assert np.array_equal(su & 15, ss & 15)
    m = np.isfinite(qu) & np.isfinite(qs) & (qu < 1e8) & ((su & (32 | 64)) == 0)
    assert m.mean() > 0.98
    assert _logq_ok(qs[m], qu[m]).all()
    assert np.allclose(to_np(rs["tw"]), to_np(ru["tw"]), atol=TOL_TW, equal_nan=True)


def test_stretched_and_uniform_jobs_in_one_batch(fq):
    """A stretched cube and a uniform one in one persistent launch: each map equals
    its own call's (the uniform job alone takes the single-job kernel, so the two
    agree to the tracing tolerance, not bit for bit)."""
    import torch

    ws = synth.config_c1s(1, nseed=48)
    wu = synth.config_c1(2, nseed=40)
    _say("batch: stretched c1s + uniform c1")
    dev = [(_dev(ws.field), ws.grid, ws.plane), (_dev(wu.field), wu.grid, wu.plane)]
    rb = fq.q2d_batch(dev, fq.Params(), want_lines=False)
    torch.cuda.synchronize()
    for (B, g, pl), r in zip(dev, rb):
        r1 = fq.q2d(B, g, pl, fq.Params())
        torch.cuda.synchronize()
        a, b = to_np(r["q"]).ravel(), to_np(r1["q"]).ravel()
        m = np.isfinite(a) & np.isfinite(b) & (b < 1e8)
        assert np.array_equal(np.isfinite(a), np.isfinite(b))
        assert _logq_ok(a[m], b[m]).all()
        assert np.allclose(to_np(r["tw"]), to_np(r1["tw"]), atol=TOL_TW, equal_nan=True)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_stretched_q3d_matches_oracle(fq, prec):
    """3-D maps (rotated S0 where |Bz/B| < 0.05) on a stretched charge cube."""
    import torch

    rng = np.random.default_rng(4)
    x = synth.clustered_axis(33, 0.0, 1.0, 0.45, 1.3)
    z = synth.geometric_axis(25, 0.0, 0.75, 1.04)
    g = synth.stretched_grid(x, x.copy(), z)
    pos, q = synth.draw_charges(rng, 6)
    B = synth.charges_field(g, pos, q)
    vx = synth.Voxels((1 / 32, 1 / 32, 0.75 / 20), (1 / 16, 1 / 16, 0.75 / 10), (15, 15, 9))
    _say(f"stretched q3d 15x15x9 voxels, precision {prec}")
    o = oracle.q3d(B, g, vx, ORC_TOL)
    r = fq.q3d(_dev(B), g, vx, fq.Params(precision=prec), want_lines=True)
    torch.cuda.synchronize()
    print(compare_maps(r, o, f"q3d-stretched-{prec}"))


def test_malformed_node_coordinates(fq):
    """Node coordinates that are not strictly increasing, or that do not span the
    box that origin and spacing give, mark every line FQ_ST_NONFINITE; Method II
    on a stretched grid is refused."""
    g = _random_stretched(9, 9, 11, seed=9)
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    pl = Plane((0.1, 0.1, 0.0), (1, 0, 0), (0, 1, 0), 4, 4, 0.2, 0.2)
    z = g.coord(2).copy()
    z[4], z[5] = z[5], z[4]
    bad = synth.Grid(g.nx, g.ny, g.nz, g.origin, g.spacing, (g.coord(0), g.coord(1), z))
    _say("non-increasing z nodes")
    r = _q2d(fq, B, bad, pl, F64)
    assert np.all(to_np(r["status"]) & fq.ST_NONFINITE)
    short = synth.Grid(g.nx, g.ny, g.nz, g.origin, (g.spacing[0], g.spacing[1], g.spacing[2] * 1.1),
                       g.coords)
    _say("z nodes not spanning the box")
    r = _q2d(fq, B, short, pl, F32X)
    assert np.all(to_np(r["status"]) & fq.ST_NONFINITE)
    _say("method II on a stretched grid")
    with pytest.raises(ValueError, match="unsupported"):
        _q2d(fq, B, g, pl, F64, method=1)


def test_in_flight_form_equals_default_on_a_stretched_grid(fq, c1s):
    """The F32X map with in_flight set (its FP64 pass at three waves per SIMD, the
    list longest first) equals the default one bit for bit on the stretched cube."""
    import torch

    w, _ = c1s
    _say("c1s in_flight form")
    a = fq.q2d(_dev(w.field), w.grid, w.plane, fq.Params(precision=F32X), want_lines=True)
    b = fq.q2d(_dev(w.field), w.grid, w.plane, fq.Params(precision=F32X, in_flight=True), want_lines=True)
    torch.cuda.synchronize()
    for k in ("q", "tw", "length", "status"):
        assert np.array_equal(to_np(a[k]), to_np(b[k]), equal_nan=True), k
    for k in ("end_b", "end_f"):
        assert np.array_equal(to_np(a["lines"][k]), to_np(b["lines"][k]), equal_nan=True), k
