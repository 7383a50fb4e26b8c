"""Q_perp by Method I (S1, S2 rotated perpendicular to B at the line's ends, Section
2.1) and the length edge map |grad_S0 length| on the GPU, through the C-ABI, in both
forms: closed forms, and parity with the oracle's q2d_perp on the charge-cube map.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import Plane, cubic_grid, linear_field

from gpu_util import LOG10_2, QMAX, TOL_LOGQ, to_np

pytestmark = pytest.mark.gpu

F32X, F64 = 0, 1

# The length edge map differences the lengths of neighbouring lines over the seed
# spacing d: length errors e (about 1e-7 of the box in FP64-accurate lines) enter as
# e / d, and the map's own scale grows with Q. Bar: 1e-4 absolute, or 1e-4 relative
# where the edge exceeds 1.
TOL_EDGE = 1e-4


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


def _map(fq, B, g, pl, prec, method=0):
    import torch

    r = fq.q2d(torch.from_numpy(np.ascontiguousarray(B)).cuda(), g, pl,
               fq.Params(precision=prec, method=method), perp=True)
    torch.cuda.synchronize()
    return {k: to_np(v) for k, v in r.items() if k in ("q", "qperp", "fledge", "status", "length")}


def _logq_ok(got, exp):
    le = np.log10(np.asarray(exp, float))
    return np.abs(np.log10(np.asarray(got, float)) - le) / np.maximum(np.abs(le), LOG10_2) <= TOL_LOGQ


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_perp_closed_forms(fq, prec):
    """Uniform field: Q_perp = 2, no edge. Tilted field ending on the side face x+:
    Q = r + 1/r there but Q_perp = 2 and the edge is |B| / bx. Sheared field:
    Q_perp = 2 + s^2 / (1 + a^2) and the edge s |a| / sqrt(1 + a^2)."""
    g = cubic_grid(17, 17, 17)
    _say(f"perp uniform, precision {prec}")
    r = _map(fq, linear_field(g, np.zeros((3, 3)), [0, 0, 1]), g, synth.plane_z0(8), prec)
    assert np.allclose(r["qperp"], 2.0, rtol=1e-6) and np.allclose(r["fledge"], 0.0, atol=TOL_EDGE)
    bx, bz = 2.0, 1.0
    pl = synth.plane_z0(20)
    _say(f"perp tilted, precision {prec}")
    r = _map(fq, linear_field(g, np.zeros((3, 3)), [bx, 0, bz]), g, pl, prec)
    inner = (np.abs(r["q"] / (bz / bx + bx / bz) - 1) < 1e-6) & ((r["status"] & (16 | 32)) == 0)
    assert inner.sum() > 20
    assert _logq_ok(r["qperp"][inner], 2.0).all()
    assert np.allclose(r["fledge"][inner], math.hypot(bx, bz) / bx, rtol=TOL_EDGE)
    s, y0 = 0.5, 0.5
    pl = Plane((0.41, 0.25, 0.0), (1, 0, 0), (0, 1, 0), 5, 5, 0.01, 0.01)
    _say(f"perp sheared, precision {prec}")
    r = _map(fq, linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1]), g, pl, prec)
    a = (s * (pl.points()[:, 1] - y0)).reshape(5, 5)
    assert _logq_ok(r["qperp"], 2 + s * s / (1 + a * a)).all()
    inn = (slice(1, -1), slice(1, -1))
    assert np.allclose(r["fledge"][inn], (np.abs(s * a) / np.sqrt(1 + a * a))[inn], atol=TOL_EDGE)


@pytest.fixture(scope="module")
def c1_perp():
    w = synth.config_c1(0)
    return w, oracle.q2d_perp(w.field, w.grid, w.plane, {"tol": 1e-10})


@pytest.mark.parametrize("prec,method", [(F32X, 0), (F64, 0), (F64, 1)],
                         ids=["f32x", "f64", "f64-method2"])
def test_c1_perp_parity(fq, c1_perp, prec, method):
    """The 128 x 128 map of the 4-charge cube: Method I Q_perp and the length edge
    map against the oracle's at every point where both succeed, no stencil line ends
    near a box edge and Q_perp < 1e8 (Method II: the same edge map from its lines'
    lengths; its own Q_perp is compared with the oracle's Method II elsewhere)."""
    w, o = c1_perp
    _say(f"c1 perp map, precision {prec}, method {method}")
    r = _map(fq, w.field, w.grid, w.plane, prec, method)
    bad = oracle.FATAL | oracle.ORC_EDGE | oracle.ORC_MIXEDFACE
    st = r["status"].astype(np.uint16) | o["status"].astype(np.uint16)
    m = ((st & bad) == 0) & np.isfinite(o["qperp"]) & (o["qperp"] < QMAX)
    assert m.mean() > 0.9
    if method == 0:
        ok = _logq_ok(r["qperp"][m], o["qperp"][m])
        print("qperp: points", int(m.sum()), "over", int((~ok).sum()))
        assert ok.all(), (np.flatnonzero(~ok)[:5], r["qperp"][m][~ok][:5], o["qperp"][m][~ok][:5])
    d = np.abs(r["fledge"][m] - o["fledge"][m])
    lim = TOL_EDGE * np.maximum(1.0, o["fledge"][m])
    print("fledge: max abs", float(d.max()), "max over bar", float((d / lim).max()))
    assert (d <= lim).all()
