"""A cylindrical mapping surface (Section 3: B = (x, -y, 0) with S1, S2 on the
cylinder x^2 + y^2 = 1) on the GPU, through the C-ABI, in both forms: the paper's
closed form, a tilted uniform field, and parity with the oracle's cylinder map on
the 4-charge cube.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import linear_field

from gpu_util import TOL_FOOT, TOL_LOGQ, compare_maps, to_np

pytestmark = pytest.mark.gpu

F32X, F64 = 0, 1


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


def _qcyl(fq, B, g, cyl, prec, **kw):
    import torch

    r = fq.qcyl(torch.from_numpy(np.ascontiguousarray(B)).cuda(), g, cyl,
                fq.Params(precision=prec, **kw), want_lines=True)
    torch.cuda.synchronize()
    return r


def _box():
    return synth.Grid(31, 31, 11, (-1.5, -1.5, 0.0), (0.1, 0.1, 0.1))


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_cylinder_paper_example(fq, prec):
    """B = (x, -y, 0) on x^2 + y^2 = 1: theta1 -> pi/2 - theta1 at the same z, Q = 2,
    Tw = 0; the half pointing out of the cylinder ends at its seed (face
    FQ_FACE_CYL), the other on the cylinder."""
    g = _box()
    B = linear_field(g, [[1, 0, 0], [0, -1, 0], [0, 0, 0]], [0, 0, 0])
    cyl = synth.Cylinder((0.0, 0.0), 1.0, 0.1, 0.05, 27, 0.2, 0.1, 5)
    _say(f"cylinder paper example, precision {prec}")
    r = _qcyl(fq, B, g, cyl, prec)
    q = to_np(r["q"])
    st = to_np(r["status"]).astype(np.uint16)
    inner = (slice(1, -1), slice(1, -1))
    assert np.all(st[inner] == 0)
    assert np.all(np.abs(np.log10(q[inner]) / math.log10(2.0) - 1) <= TOL_LOGQ)
    assert np.allclose(to_np(r["tw"]), 0.0, atol=1e-9)
    L = {k: to_np(v) for k, v in r["lines"].items()}
    assert np.all(L["face_b"] == fq.FQ_FACE_CYL) and np.all(L["face_f"] == fq.FQ_FACE_CYL)
    th = cyl.theta0 + cyl.dtheta * np.arange(cyl.ntheta)
    eb = L["end_b"].reshape(cyl.nz, cyl.ntheta, 3)
    ef = L["end_f"].reshape(cyl.nz, cyl.ntheta, 3)
    seeds = cyl.points().reshape(cyl.nz, cyl.ntheta, 3)
    far = np.where((th < math.pi / 4)[None, :, None], eb, ef)
    near = np.where((th < math.pi / 4)[None, :, None], ef, eb)
    assert np.allclose(near, seeds, rtol=0, atol=1e-14)
    assert np.allclose(np.hypot(far[..., 0], far[..., 1]), 1.0, atol=TOL_FOOT)
    assert np.allclose(np.arctan2(far[..., 1], far[..., 0]), math.pi / 2 - th[None, :], atol=TOL_FOOT)
    assert np.allclose(far[..., 2], seeds[..., 2], atol=TOL_FOOT)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_cylinder_tilted_uniform_field(fq, prec):
    """B = (1, 0, bz): Q = 2 + (2 bz sin theta1 sin(d)/d)^2 on the stencil, lengths
    2 |cos theta1| sqrt(1 + bz^2), across the wrap of theta at pi."""
    g = _box()
    bz = 0.3
    B = linear_field(g, np.zeros((3, 3)), [1.0, 0.0, bz])
    cyl = synth.Cylinder((0.0, 0.0), 1.0, 2.0, 0.04, 56, 0.1, 0.02, 4)
    _say(f"cylinder tilted field, precision {prec}")
    r = _qcyl(fq, B, g, cyl, prec)
    th = cyl.theta0 + cyl.dtheta * np.arange(cyl.ntheta)
    c = 2 * bz * np.sin(th) * math.sin(cyl.dtheta) / cyl.dtheta
    q = to_np(r["q"])[1:-1, 1:-1]
    qexp = np.broadcast_to(2 + c * c, to_np(r["q"]).shape)[1:-1, 1:-1]
    assert np.all(np.abs(np.log10(q) / np.log10(qexp) - 1) <= TOL_LOGQ)
    lexp = np.broadcast_to(2 * np.abs(np.cos(th)) * math.sqrt(1 + bz * bz), to_np(r["length"]).shape)
    assert np.allclose(to_np(r["length"]), lexp, atol=1e-6)


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
def test_cylinder_charge_cube_parity(fq, prec):
    """A cylinder (centre (0.5, 0.5), radius 0.3, z 0.05-0.85) in the 4-charge 64^3
    cube: Q, Tw, footpoints and statuses against the oracle's cylinder map at every
    point (lines that leave through the box's faces included)."""
    w = synth.config_c1(0)
    cyl = synth.Cylinder((0.5, 0.5), 0.3, 0.0, 2 * math.pi / 96, 96, 0.05, 0.8 / 24, 25)
    _say(f"cylinder in the charge cube, precision {prec}")
    o = oracle.qcyl(w.field, w.grid, cyl, {"tol": 1e-10})
    r = _qcyl(fq, w.field, w.grid, cyl, prec)
    ob = {"q": o["q"], "tw": o["tw"], "status": o["status"], "lines": o["lines"]}
    gb = {"q": to_np(r["q"]).ravel(), "tw": to_np(r["tw"]).ravel(),
          "status": to_np(r["status"]).astype(np.uint16).ravel(),
          "lines": {k: to_np(r["lines"][k]) for k in ("end_b", "end_f", "face_b", "face_f")}}
    st = compare_maps(gb, ob, f"cyl-{prec}", raw=True)
    print(st)
    assert st["excluded_frac"] < 0.1
