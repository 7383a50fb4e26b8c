"""Method II (Section 2.1, Eq. rb2, Eq. q_scott) on the GPU, through the C-ABI, in
both forms: closed forms of Q and Q_perp, and parity with the oracle's Method II
on a charge-field map and a 3-D map.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import Plane, cubic_grid, linear_field

from gpu_util import LOG10_2, QMAX, TOL_LOGQ, compare_maps, to_np

pytestmark = pytest.mark.gpu

F32X, F64 = 0, 1
M2 = 1


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


def _logq_ok(got, exp):
    got = np.asarray(got, float)
    exp = np.asarray(exp, float)
    le = np.log10(exp)
    return np.abs(np.log10(got) - le) / np.maximum(np.abs(le), LOG10_2) <= TOL_LOGQ


def _map(fq, B, g, pl, prec, tol=0.0):
    import torch

    r = fq.q2d(_dev(B), g, pl, fq.Params(precision=prec, method=M2, tol_perp=tol), want_lines=True)
    torch.cuda.synchronize()
    return r


# Method II's S0 is perpendicular to B, so Eq. tol gives its lines the per-step bound
# tol_perp itself, without the angle factor that tightens it for Method I's seeds on
# an inclined plane. Its product is Q from U and V, not the footpoints: at the
# default bound Q, Q_perp and Tw are compared, and the footpoints at 1e-7, where the
# bound is as tight as Method I's for these planes.
FOOT_TOL_PERP = 1e-7


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_m2_closed_forms(fq, prec):
    """Uniform field: Q = Q_perp = 2. Tilted uniform field to the side face x+:
    Q = r + 1/r, Q_perp = 2. Sheared field: Q = 2 + s^2, Q_perp = 2 + s^2/(1 + a^2).
    Hyperbolic field: Q = 2 cosh 2kL (kL = 2 and 4)."""
    g = cubic_grid(17, 17, 17)
    pl = Plane((0.3, 0.35, 0.0), (1, 0, 0), (0, 1, 0), 4, 3, 0.05, 0.1)
    _say(f"m2 uniform, precision {prec}")
    r = _map(fq, linear_field(g, np.zeros((3, 3)), [0, 0, 1]), g, pl, prec)
    assert np.all(to_np(r["status"]) == 0)
    assert np.allclose(to_np(r["q"]), 2.0, rtol=1e-6) and np.allclose(to_np(r["qperp"]), 2.0, rtol=1e-6)
    bx, bz = 2.0, 1.0
    pl = Plane((0.62, 0.3, 0.0), (1, 0, 0), (0, 1, 0), 4, 3, 0.05, 0.1)
    _say(f"m2 tilted, precision {prec}")
    r = _map(fq, linear_field(g, np.zeros((3, 3)), [bx, 0, bz]), g, pl, prec)
    assert np.all(to_np(r["lines"]["face_f"]) == 1)
    assert _logq_ok(to_np(r["q"]), bz / bx + bx / bz).all()
    assert _logq_ok(to_np(r["qperp"]), 2.0).all()
    s, y0 = 0.5, 0.5
    pl = Plane((0.45, 0.3, 0.0), (1, 0, 0), (0, 1, 0), 1, 5, 0.1, 0.1)
    _say(f"m2 sheared, precision {prec}")
    r = _map(fq, linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1]), g, pl, prec)
    a = s * (pl.points()[:, 1] - y0)
    assert _logq_ok(to_np(r["q"]).ravel(), 2 + s * s).all()
    assert _logq_ok(to_np(r["qperp"]).ravel(), 2 + s * s / (1 + a * a)).all()
    for kL in (2.0, 4.0):
        B = linear_field(g, [[kL, 0, 0], [0, -kL, 0], [0, 0, 0]], [-kL * 0.5, kL * 0.5, 1])
        pl = Plane((0.5 + 0.05 * math.exp(-kL), 0.52, 0.0), (1, 0, 0), (0, 1, 0), 1, 1, 0.1, 0.1)
        _say(f"m2 hyperbolic kL {kL}, precision {prec}")
        r = _map(fq, B, g, pl, prec)
        assert _logq_ok(to_np(r["q"]).ravel(), 2 * math.cosh(2 * kL)).all(), (to_np(r["q"]), kL)


def _compare_qperp(gq, oq, gst, ost, label):
    bad = oracle.FATAL | oracle.ORC_EDGE
    m = (((gst | ost) & bad) == 0) & np.isfinite(oq) & (oq < QMAX)
    assert m.mean() > 0.9
    ok = _logq_ok(gq[m], oq[m])
    assert ok.all(), (label, np.flatnonzero(~ok)[:5], gq[m][~ok][:5], oq[m][~ok][:5])


def _gpu_block(r):
    return {"q": to_np(r["q"]).ravel(), "tw": to_np(r["tw"]).ravel(),
            "status": to_np(r["status"]).astype(np.uint16).ravel(),
            "lines": {k: to_np(r["lines"][k]) for k in ("end_b", "end_f", "face_b", "face_f")}}


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_m2_c1_map_parity(fq, prec):
    """The 128 x 128 Method II map of the 4-charge 64^3 cube against the oracle's
    Method II (offset differences of B/B), every point: Q, Q_perp and Tw at the
    default bound, footpoints too at tol_perp 1e-7."""
    w = synth.config_c1(0)
    seeds = w.plane.points()
    o = oracle.method2(w.field, w.grid, seeds, 2, {"tol": 1e-10})
    ob = {"q": o["q"], "tw": o["tw"], "status": o["status"], "lines": o["lines"]}
    for tol in (0.0, FOOT_TOL_PERP):
        _say(f"m2 c1 map, precision {prec}, tol_perp {tol or 'default'}")
        r = _map(fq, w.field, w.grid, w.plane, prec, tol)
        gb = _gpu_block(r)
        print(compare_maps(gb, ob, f"m2-c1-{prec}-{tol}", foot=tol > 0, raw=True))
        _compare_qperp(to_np(r["qperp"]).ravel(), o["qperp"], gb["status"], o["status"], "qperp")


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_m2_q3d_parity(fq, prec):
    """Method II at the voxel centres of a small charge cube (one line per voxel;
    S0 perpendicular to B everywhere, so no rotated extras) against the oracle."""
    import torch

    rng = np.random.default_rng(2)
    g = cubic_grid(33, 33, 25)
    pos, q = synth.draw_charges(rng, 6)
    B = synth.charges_field(g, pos, q)
    ux, uy, uz = g.upper
    vx = synth.Voxels((ux / 32, uy / 32, uz / 20), (ux / 16, uy / 16, uz / 10), (15, 15, 9))
    o = oracle.method2(B, g, vx.points(), 2, {"tol": 1e-10})
    ob = {"q": o["q"], "tw": o["tw"], "status": o["status"], "lines": o["lines"]}
    Bd = _dev(B)
    for tol in (0.0, FOOT_TOL_PERP):
        _say(f"m2 q3d 15x15x9 voxels, precision {prec}, tol_perp {tol or 'default'}")
        r = fq.q3d(Bd, g, vx, fq.Params(precision=prec, method=M2, tol_perp=tol), want_lines=True)
        torch.cuda.synchronize()
        gb = _gpu_block(r)
        assert not (gb["status"] & fq.ST_ROTATED).any()
        print(compare_maps(gb, ob, f"m2-q3d-{prec}-{tol}", foot=tol > 0, raw=True))
        _compare_qperp(to_np(r["qperp"]).ravel(), o["qperp"], gb["status"], o["status"], "q3d qperp")
