"""The fixed-step RK4 schemes (classic and Kutta's 3/8 rule, Section 2.3) on the GPU,
through the C-ABI: their end points converge to the oracle's at fourth order as
the step shrinks, and at a small step the maps meet the parity bar in both forms.

Every case prints what it runs before touching the GPU, so a failing run names it.
"""

import sys

import numpy as np
import pytest

import oracle
import synth

from gpu_util import compare_maps, to_np

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


@pytest.fixture(scope="module")
def c1():
    w = synth.config_c1(0)
    rng = np.random.default_rng(4)
    seeds = np.concatenate([rng.uniform(0.1, 0.9, (200, 3)),
                            np.c_[rng.uniform(0.1, 0.9, (100, 2)), np.zeros(100)]])
    o = oracle.trace(w.field, w.grid, seeds, opts={"tol": 1e-12})
    return w, seeds, o


@pytest.mark.parametrize("scheme", [1, 2], ids=["rk4", "rk4_38"])
def test_fixed_step_converges_at_fourth_order(fq, scheme):
    """All-FP64 lines of the hyperbolic field B = (k(x - xc), -k(y - yc), 1) from the
    bottom to the top face, x2 - xc = (x1 - xc) e^{kL}, y2 - yc = (y1 - yc) e^{-kL}
    (Eq. rb), at fixed steps of 0.4, 0.2 and 0.1 grid spacings: the end error falls
    by about 2^4 per halving."""
    import math

    import torch

    from synth import cubic_grid, linear_field

    kL = 2.0
    g = cubic_grid(17, 17, 17)
    B = torch.from_numpy(linear_field(g, [[kL, 0, 0], [0, -kL, 0], [0, 0, 0]],
                                      [-kL * 0.5, kL * 0.5, 1])).cuda()
    rng = np.random.default_rng(2)
    seeds = np.c_[0.5 + rng.uniform(-0.1, 0.1, 32) * math.exp(-kL), rng.uniform(0.3, 0.7, 32),
                  np.zeros(32)]
    exp_x = 0.5 + (seeds[:, 0] - 0.5) * math.exp(kL)
    exp_y = 0.5 + (seeds[:, 1] - 0.5) * math.exp(-kL)
    errs = []
    for h in (0.4, 0.2, 0.1):
        _say(f"scheme {scheme}, fixed step {h}")
        r = fq.trace(B, g, torch.from_numpy(seeds).cuda(),
                     params=fq.Params(precision=F64, scheme=scheme, step_perp=h, step_min=h))
        torch.cuda.synchronize()
        assert np.all(to_np(r["face_f"]) == 5)
        e = to_np(r["end_f"])
        errs.append(max(np.abs(e[:, 0] - exp_x).max(), np.abs(e[:, 1] - exp_y).max()))
    print(scheme, errs)
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs


@pytest.mark.parametrize("scheme", [1, 2], ids=["rk4", "rk4_38"])
def test_fixed_step_ends_on_a_charge_field(fq, c1, scheme):
    """Lines of the 4-charge 64^3 cube (interior seeds and seeds on the bottom face,
    arcades included) at a fixed step of 0.1 grid spacings end within 1e-7 box units
    of the oracle's (FP64)."""
    import torch

    w, seeds, o = c1
    _say(f"scheme {scheme}, charge field ends")
    r = fq.trace(torch.from_numpy(w.field).cuda(), w.grid, torch.from_numpy(seeds).cuda(),
                 params=fq.Params(precision=F64, scheme=scheme, step_perp=0.1, step_min=0.1))
    torch.cuda.synchronize()
    st = to_np(r["status"]).astype(np.uint16)
    ok = ((st | o["status"]) & (oracle.FATAL | oracle.ORC_EDGE)) == 0
    assert ok.mean() > 0.9
    for k in ("face_b", "face_f"):
        assert np.array_equal(to_np(r[k])[ok], o[k][ok])
    e = max(np.abs(to_np(r[k]) - o[k]).max(axis=1)[ok].max() for k in ("end_b", "end_f"))
    assert e < 1e-7, e


@pytest.mark.parametrize("prec", [F32X, F64], ids=["f32x", "f64"])
@pytest.mark.parametrize("scheme", [1, 2], ids=["rk4", "rk4_38"])
def test_fixed_step_map_parity(fq, prec, scheme):
    """The full 128 x 128 C1 map with a fixed step of 0.1 grid spacings, against the
    oracle with the parity mask and tolerances of every other map test."""
    import torch

    w = synth.config_c1(0)
    _say(f"c1 map, scheme {scheme}, precision {prec}")
    r = fq.q2d(torch.from_numpy(w.field).cuda(), w.grid, w.plane,
               fq.Params(precision=prec, scheme=scheme, step_perp=0.1, step_min=0.1),
               want_lines=True)
    torch.cuda.synchronize()
    o = oracle.q2d(w.field, w.grid, w.plane, {"tol": 1e-10})
    print(compare_maps(r, o, f"c1-scheme{scheme}-{prec}"))


@pytest.mark.parametrize("scheme", [1, 2], ids=["rk4", "rk4_38"])
def test_recorded_fixed_step_map_equals_q2d(fq, scheme):
    """The adjoint's checkpointed forward pass of a fixed-step scheme writes the map of
    fastqsl_q2d bit for bit (the gradient itself is checked with the adjoint)."""
    import torch

    w = synth.config_c1(0)
    B = torch.from_numpy(w.field).cuda()
    p = fq.Params(precision=F64, scheme=scheme, step_perp=0.1, step_min=0.1)
    _say(f"recorded map, scheme {scheme}")
    rec = fq.q2d_record(B, w.grid, w.plane, p, 16)
    ref = fq.q2d(B, w.grid, w.plane, p)
    torch.cuda.synchronize()
    for k in ("q", "tw", "length", "status"):
        assert np.array_equal(to_np(rec[k]), to_np(ref[k]), equal_nan=True), k
