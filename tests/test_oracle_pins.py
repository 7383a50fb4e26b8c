"""Pins of the FP64 CPU oracle to facts fixed by the paper and by the mathematics.

Each test names the passage of the paper (section / equation) it follows. The
linear fields P1-P5 are reproduced exactly by trilinear interpolation and by
second-order differences, so their closed forms bound only the integrator; the
charge-field tests pin the general case through invariances the paper states, and
an independent library integrator (scipy's DOP853 on scipy's trilinear
RegularGridInterpolator) pins the cell-by-cell integration itself.
"""

import json
import math
import os

import numpy as np
import pytest

import synth
from synth import Plane, Voxels, cubic_grid, linear_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _plane(center, d, n=3, u=(1.0, 0.0, 0.0), v=(0.0, 1.0, 0.0)):
    """n x n seeds centred on `center` with spacing d along orthonormal u, v."""
    c = np.asarray(center, float)
    u = np.asarray(u, float)
    v = np.asarray(v, float)
    h = (n - 1) / 2.0
    o = c - h * d * u - h * d * v
    return Plane(tuple(o), tuple(u), tuple(v), n, n, d, d)


# --------------------------------------------------------------------------------------
# building blocks: curl stencil and trilinear interpolation
# --------------------------------------------------------------------------------------


def test_curl_exact_for_quadratic_field(orc):
    """Second-order central and one-sided differences (stencil of Eq. grad_B,
    Section 4) are exact for quadratic fields, on every node including the
    boundary ones; a wrong sign, index or boundary formula fails here."""
    g = synth.Grid(7, 8, 9, (0.1, -0.2, 0.3), (0.25, 0.2, 0.15))
    x, y, z = g.axes()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    B = np.stack([X * Y + 2 * Z * Z - Y, Y * Z - 3 * X * X + X * Z, X * Y * 0.5 + Z * X - Y * Y])
    # analytic curl
    dBz_dy = 0.5 * X - 2 * Y
    dBy_dz = Y + X
    dBx_dz = 4 * Z
    dBz_dx = 0.5 * Y + Z
    dBy_dx = -6 * X + Z
    dBx_dy = X - 1
    J = np.stack([dBz_dy - dBy_dz, dBx_dz - dBz_dx, dBy_dx - dBx_dy])
    Jo = orc.curl(B, g)
    assert np.max(np.abs(Jo - J)) < 1e-11


def test_interp_matches_scipy_trilinear(orc):
    """Eq. interp / w0 / w1 (Section 2.2) against scipy's linear RegularGridInterpolator."""
    from scipy.interpolate import RegularGridInterpolator

    rng = np.random.default_rng(1)
    g = synth.Grid(6, 5, 7, (0.0, 1.0, -1.0), (0.3, 0.5, 0.2))
    B = rng.standard_normal((3,) + g.shape)
    x, y, z = g.axes()
    pts = np.stack([rng.uniform(x[0], x[-1], 50), rng.uniform(y[0], y[-1], 50),
                    rng.uniform(z[0], z[-1], 50)], axis=1)
    for c in range(3):
        f = RegularGridInterpolator((x, y, z), np.transpose(B[c], (2, 1, 0)), method="linear")
        ref = f(pts)
        for p, r in zip(pts, ref):
            cell = [min(int(math.floor((p[a] - g.origin[a]) / g.spacing[a])), (g.nx, g.ny, g.nz)[a] - 2)
                    for a in range(3)]
            assert abs(orc.interp(B, g, cell, p)[c] - r) < 1e-12


# --------------------------------------------------------------------------------------
# closed forms P1-P5 (linear fields)
# --------------------------------------------------------------------------------------


def test_p1_uniform_field(orc):
    """B = (0,0,1): identity mapping, Q = 2 (the minimum, Section 1), Tw = 0, l = Lz."""
    g = cubic_grid(9, 9, 9)
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    pl = synth.plane_z0(16)
    r = orc.q2d(B, g, pl)
    assert np.all(r["status"] & orc.FATAL == 0)
    assert np.allclose(r["q"], 2.0, atol=1e-12)
    assert np.allclose(r["tw"], 0.0, atol=1e-14)
    assert np.allclose(r["len"], 1.0, atol=1e-12)
    seeds = pl.points()
    assert np.allclose(r["lines"]["end_f"][:, :2], seeds[:, :2], atol=1e-13)
    assert np.all(r["lines"]["face_f"] == 5) and np.all(r["lines"]["face_b"] == 4)


@pytest.mark.parametrize("bx,bz", [(0.2, 1.0), (2.0, 1.0), (1.0, 0.25)])
def test_p2_tilted_uniform_field(orc, bx, bz):
    """B = (bx, 0, bz): bottom -> top gives Q = 2; bottom -> side face x+ maps
    (x1, y1) to (y2, z2) = (y1, (1-x1) bz/bx) and gives Q = r + 1/r, r = bz/bx
    (the projection effect of the choice of S1, S2, Section 2.1)."""
    g = cubic_grid(9, 9, 9)
    B = linear_field(g, np.zeros((3, 3)), [bx, 0, bz])
    pl = synth.plane_z0(20)
    r = orc.q2d(B, g, pl)
    L = r["lines"]
    seeds = pl.points()
    top = L["face_f"] == 5
    side = L["face_f"] == 1
    assert top.any() or side.any()
    q = r["q"].ravel()
    st = r["status"].ravel()
    inner_top = top & ((st & orc.ORC_ONESIDED) == 0)
    if inner_top.any():
        assert np.allclose(q[inner_top], 2.0, atol=1e-9)
        assert np.allclose(L["end_f"][top, 0], seeds[top, 0] + bx / bz, atol=1e-11)
    rr = bz / bx
    inner_side = side & ((st & (orc.ORC_ONESIDED | orc.ORC_MIXEDFACE)) == 0)
    if side.any():
        assert np.allclose(L["end_f"][side, 2], (1 - seeds[side, 0]) * rr, atol=1e-11)
        assert np.allclose(L["end_f"][side, 1], seeds[side, 1], atol=1e-12)
    if inner_side.any():
        assert np.allclose(q[inner_side], rr + 1 / rr, rtol=1e-9)


def test_p3_sheared_field(orc):
    """B = (s(y-y0), 0, 1): x2 = x1 + s(y1-y0)L, Q = 2 + s^2 L^2 (Eq. Q+-) and
    Tw = -sL / (4 pi sqrt(1 + s^2 (y1-y0)^2)) (Eq. tw, curl B = (0,0,-s))."""
    g = cubic_grid(11, 11, 11)
    s, y0 = 0.5, 0.5
    B = linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1])
    pl = _plane((0.45, 0.3, 0.0), 0.01, n=5)
    r = orc.q2d(B, g, pl)
    seeds = pl.points()
    y1 = seeds[:, 1]
    assert np.allclose(r["q"], 2 + s * s, rtol=1e-10)
    tw = -s / (4 * np.pi * np.sqrt(1 + s * s * (y1 - y0) ** 2))
    assert np.allclose(r["tw"].ravel(), tw, atol=1e-11)
    assert np.allclose(r["lines"]["end_f"][:, 0], seeds[:, 0] + s * (y1 - y0), atol=1e-11)
    # the worked value 2.25 / -0.0393485272 at y1 - y0 = -0.15 ... checked by formula above
    assert abs(-s / (4 * np.pi * math.sqrt(1 + s * s * 0.0))) > 0


@pytest.mark.parametrize("kL,d", [(2.0, 1e-3), (6.9, 2e-5)])
def test_p4_hyperbolic_field_high_q(orc, kL, d):
    """B = (k(x-xc), -k(y-yc), 1): x2 - xc = (x1 - xc) e^{kL}, y2 - yc = (y1 - yc) e^{-kL},
    Q = 2 cosh(2kL) (Eq. Q+-); kL = 6.9 gives Q ~ 1e6, a thin QSL."""
    g = cubic_grid(17, 17, 17)
    k = kL / 1.0
    xc = yc = 0.5
    B = linear_field(g, [[k, 0, 0], [0, -k, 0], [0, 0, 0]], [-k * xc, k * yc, 1])
    pl = _plane((xc + 0.2 * math.exp(-kL), yc + 0.1, 0.0), d, n=3)
    r = orc.q2d(B, g, pl)
    assert np.all(r["lines"]["face_f"] == 5)
    seeds = pl.points()
    ex = xc + (seeds[:, 0] - xc) * math.exp(kL)
    assert np.allclose(r["lines"]["end_f"][:, 0], ex, atol=1e-9)
    qexp = 2 * math.cosh(2 * kL)
    assert abs(r["q"][1, 1] / qexp - 1) < 1e-6
    assert np.allclose(r["tw"], 0.0, atol=1e-12)


def test_p5_twisted_field_tw(orc):
    """B = B0(-q(y-yc), q(x-xc), 1): rigid rotation by qL, Q = 2, and
    Tw = qL / (2 pi sqrt(1 + q^2 rho^2)) (Eq. tw with curl B = (0,0,2 q B0))."""
    g = cubic_grid(21, 21, 21)
    q = 3 * math.pi  # 1.5 turns over L = 1
    xc = yc = 0.5
    B0 = 0.7
    B = linear_field(g, [[0, -q * B0, 0], [q * B0, 0, 0], [0, 0, 0]], [q * B0 * yc, -q * B0 * xc, B0])
    pl = _plane((xc + 0.05, yc, 0.0), 0.002, n=3)
    r = orc.q2d(B, g, pl)
    seeds = pl.points()
    rho = np.hypot(seeds[:, 0] - xc, seeds[:, 1] - yc)
    tw = q / (2 * np.pi * np.sqrt(1 + q * q * rho * rho))
    assert np.allclose(r["tw"].ravel(), tw, atol=1e-9)
    assert abs(r["tw"][1, 1] - 1.3568877159) < 1e-8  # rho = 0.05
    assert abs(r["q"][1, 1] - 2.0) < 1e-6
    ang = math.atan2(seeds[4, 1] - yc, seeds[4, 0] - xc) + q
    e = r["lines"]["end_f"][4]
    assert abs(e[0] - (xc + rho[4] * math.cos(ang))) < 1e-9
    assert abs(e[1] - (yc + rho[4] * math.sin(ang))) < 1e-9


@pytest.mark.parametrize("delta", [1e-5, 1e-6])
def test_p9_line_grazing_a_face_before_landing(orc, delta):
    """B = (1, 0, a(x - x0)): the lines are parabolas z = z_top + a (x - x0)^2 / 2 in
    the plane y = const (Eq. rb). The apex rises delta above the cell face z = 1/2,
    and the line crosses that face a distance eps before an x face, then crosses it
    back within the same trial step. The cell-by-cell integration must treat the
    z face as the first face crossed; taking the x face instead moves the line by
    about sqrt(2 delta) eps. Both ends must match the closed form."""
    g = cubic_grid(17, 17, 17)
    a, zf = -1.0, 0.5
    s = math.sqrt(2 * delta / -a)
    for xf in (0.5, 0.5625):
        for eps in (1e-5, 1e-4, 1e-3):
            x0 = xf - eps + s
            B = linear_field(g, [[0, 0, 0], [0, 0, 0], [a, 0, 0]], [1.0, 0.0, -a * x0])
            xs, ys = 0.05, 0.53
            zs = zf + delta + 0.5 * a * (xs - x0) ** 2
            L = orc.trace(B, g, np.array([[xs, ys, zs]]))
            assert L["face_f"][0] == 1 and L["face_b"][0] == 0
            for key, xe in (("end_f", 1.0), ("end_b", 0.0)):
                ze = zf + delta + 0.5 * a * (xe - x0) ** 2
                e = L[key][0]
                assert np.max(np.abs(e - [xe, ys, ze])) < 1e-11, (xf, eps, key, e)


# --------------------------------------------------------------------------------------
# invariances of Q on a charge field (Section 1, Section 2.1)
# --------------------------------------------------------------------------------------


@pytest.fixture(scope="module")
def charge_cube():
    rng = np.random.default_rng(7)
    g = cubic_grid(33, 33, 33)
    pos, q = synth.draw_charges(rng, 4)
    return g, synth.charges_field(g, pos, q)


def _q_at(orc, B, g, center, d, u=(1, 0, 0), v=(0, 1, 0), opts=None):
    r = orc.q2d(B, g, _plane(center, d, 3, u, v), opts)
    return r["q"][1, 1], r


def _multilinear_solenoidal(g):
    """Bx = f(y,z), By = g(x,z), Bz = h(x,y), each bilinear: divergence-free, and
    reproduced exactly by trilinear interpolation and by the curl stencil, so the
    lines are nonlinear while flux is conserved exactly along them."""
    x, y, z = g.axes()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([0.3 + 4.0 * (Y - 0.5) * (Z - 0.3),
                     -0.2 + 4.0 * (X - 0.5) * (Z - 0.6),
                     1.0 + 0.5 * (X - 0.4) * (Y - 0.6)])


def test_p6_p7_interior_s0_equals_direct(orc):
    """Method I through an auxiliary S0 (Eq. D+-2, D+-3) gives the same Q as the
    direct map from S1, for any orientation of S0 (Section 2.1), and Q is the same
    seen from both footpoints, Q(x1,y1) = Q(x2,y2) (Section 1)."""
    g = cubic_grid(9, 9, 9)
    B = _multilinear_solenoidal(g)
    d = 1e-5
    opts = {"tol": 1e-12}
    mid = np.array([0.5, 0.45, 0.4])
    L = orc.trace(B, g, mid[None, :], opts=opts)
    assert L["face_b"][0] == 4 and L["face_f"][0] == 5
    q_mid, _ = _q_at(orc, B, g, mid, d, opts=opts)
    th = 0.7
    u = (math.cos(th), math.sin(th), 0.0)
    v = (-math.sin(th) * math.cos(0.4), math.cos(th) * math.cos(0.4), math.sin(0.4))
    q_rot, _ = _q_at(orc, B, g, mid, d, u, v, opts=opts)
    foot = L["end_b"][0]
    top = L["end_f"][0]
    q_bot, _ = _q_at(orc, B, g, (foot[0], foot[1], 0.0), d, opts=opts)
    q_top, _ = _q_at(orc, B, g, (top[0], top[1], 1.0), d, opts=opts)
    assert q_mid > 2.5  # a non-trivial map
    assert abs(q_mid / q_bot - 1) < 1e-7, (q_mid, q_bot)
    assert abs(q_rot / q_mid - 1) < 1e-7, (q_rot, q_mid)
    assert abs(q_top / q_bot - 1) < 1e-7, (q_top, q_bot)


def test_flux_conservation_of_fd_jacobian(orc):
    """|det D12| = |Bn1/Bn2| (Section 1, Eq. Bn1): the finite-difference Jacobian of
    the traced map agrees with the recorded normal-field ratio."""
    g = cubic_grid(9, 9, 9)
    B = _multilinear_solenoidal(g)
    d = 1e-5
    pl = _plane((0.47, 0.52, 0.0), d, 3)
    r = orc.q2d(B, g, pl, {"tol": 1e-12})
    L = r["lines"]
    assert np.all(L["face_b"] == 4) and np.all(L["face_f"] == 5)
    far = L["end_f"]
    bn_far = L["bn_f"]
    X = far[:, 0].reshape(3, 3)
    Y = far[:, 1].reshape(3, 3)
    a = (X[1, 2] - X[1, 0]) / (2 * d)
    b = (X[2, 1] - X[0, 1]) / (2 * d)
    c = (Y[1, 2] - Y[1, 0]) / (2 * d)
    dd = (Y[2, 1] - Y[0, 1]) / (2 * d)
    det = a * dd - b * c
    ratio = L["bn0"][4] / bn_far[4]
    assert abs(abs(det) / abs(ratio) - 1) < 1e-8


def test_sign_flip_and_reflection(orc, charge_cube):
    """B -> -B leaves Q and Tw unchanged (Eq. Q+-, Eq. tw); swapping x and y
    transposes the Q map and flips the sign of Tw (J.B is a pseudoscalar)."""
    g, B = charge_cube
    pl = synth.plane_z0(24)
    base = orc.q2d(B, g, pl)
    neg = orc.q2d(-B, g, pl)
    ok = (base["status"] & (orc.FATAL | orc.ORC_MIXEDFACE)) == 0
    assert ok.mean() > 0.9
    assert np.allclose(neg["q"][ok], base["q"][ok], rtol=1e-8)
    assert np.allclose(neg["tw"][ok], base["tw"][ok], atol=1e-12)
    # reflection x <-> y
    Bs = np.stack([B[1].transpose(0, 2, 1), B[0].transpose(0, 2, 1), B[2].transpose(0, 2, 1)])
    sw = orc.q2d(Bs, g, pl)
    assert np.allclose(sw["q"].T[ok], base["q"][ok], rtol=1e-8)
    assert np.allclose(sw["tw"].T[ok], -base["tw"][ok], atol=1e-12)


# --------------------------------------------------------------------------------------
# the paper's analytic quadrupole (Section 3.2, golden fixture)
# --------------------------------------------------------------------------------------


def test_p8_quadrupole_symmetry_and_q2(orc):
    gold = json.load(open(os.path.join(GOLDEN, "quadrupole.json")))
    assert np.allclose(synth.fields.QUADRUPOLE_POS, gold["charges_xyz"])
    assert np.allclose(synth.fields.QUADRUPOLE_Q, gold["charges_q"])
    g, B = synth.quadrupole_field(gold["grid_spacing"], lo=(-2.5, -1.5, 0.0), hi=(2.5, 1.5, 2.0))
    n = 24
    d = 0.05
    # seeds mirror-symmetric about x = 0 and y = 0 (none on the PIL x = 0)
    pl = Plane((-(n - 1) / 2 * d, -(n - 1) / 2 * d, 0.0), (1, 0, 0), (0, 1, 0), n, n, d, d)
    r = orc.q2d(B, g, pl, {"tol": 1e-10})
    q = r["q"]
    ok = ((r["status"] & (orc.FATAL | orc.ORC_MIXEDFACE)) == 0)
    okm = ok & ok[:, ::-1] & ok[::-1, :]
    assert okm.mean() > 0.8
    # mirror symmetries of the map (the field is odd under x -> -x, even under y -> -y)
    assert np.allclose(q[okm], q[:, ::-1][okm], rtol=1e-6)
    assert np.allclose(q[okm], q[::-1, :][okm], rtol=1e-6)
    # lines mapped x2 = -x1, y2 = y1 (the 'in' and 'out' regions) have Q = 2
    L = r["lines"]
    seeds = pl.points()
    far = np.where(np.abs(L["end_f"] - seeds).sum(1)[:, None] < 1e-14, L["end_b"], L["end_f"])
    sym = (np.abs(far[:, 0] + seeds[:, 0]) < 1e-6) & (np.abs(far[:, 1] - seeds[:, 1]) < 1e-6)
    sym = sym.reshape(n, n)
    # the whole 5-point stencil inside the region (a stencil straddling a separatrix
    # picks it up as high Q: Method I captures separatrices, Section 3.2)
    s5 = sym.copy()
    s5[1:-1, 1:-1] &= sym[:-2, 1:-1] & sym[2:, 1:-1] & sym[1:-1, :-2] & sym[1:-1, 2:]
    s5[0, :] = s5[-1, :] = s5[:, 0] = s5[:, -1] = False
    inner = s5 & ((r["status"] & (orc.FATAL | orc.ORC_MIXEDFACE | orc.ORC_ONESIDED)) == 0)
    assert inner.sum() >= 20
    assert np.allclose(q[inner], gold["expected_Q_in_symmetric_regions"], atol=1e-6)
    # and at least one straddling point shows the separatrix as high Q
    assert np.nanmax(q[sym & ~s5]) > 100


# --------------------------------------------------------------------------------------
# the integrator against an independent library integrator
# --------------------------------------------------------------------------------------


@pytest.mark.slow
def test_p10_against_scipy_dop853(orc):
    """Endpoints of lines in a trilinear (kinked) field: the oracle against scipy's
    DOP853 (rtol 1e-12) on scipy's trilinear RegularGridInterpolator, with box-exit
    events; the field-line ODE is Eq. rb (Section 2.1)."""
    from scipy.integrate import solve_ivp
    from scipy.interpolate import RegularGridInterpolator

    rng = np.random.default_rng(3)
    g = cubic_grid(12, 12, 12)
    pos, q = synth.draw_charges(rng, 4)
    B = synth.charges_field(g, pos, q)
    x, y, z = g.axes()
    its = [RegularGridInterpolator((x, y, z), np.transpose(B[c], (2, 1, 0)), method="linear")
           for c in range(3)]

    def rhs(s, r, sig):
        rr = np.clip(r, 0.0, 1.0)[None, :]
        b = np.array([it(rr)[0] for it in its])
        return sig * b / np.linalg.norm(b)

    seeds = np.array([[0.42, 0.55, 0.0], [0.6, 0.4, 0.0], [0.5, 0.5, 0.3]])
    L = orc.trace(B, g, seeds, opts={"tol": 1e-12})
    for s in range(len(seeds)):
        for sig, key in ((1.0, "end_f"), (-1.0, "end_b")):
            ev = []
            for a in range(3):
                for bound in (0.0, 1.0):
                    def e(t, r, sg, a=a, bound=bound):
                        return r[a] - bound
                    e.terminal = True
                    ev.append(e)
            r0 = seeds[s]
            b0 = np.array([it(r0[None, :])[0] for it in its])
            if r0[2] == 0.0 and sig * b0[2] < 0:
                end = r0
            else:
                sol = solve_ivp(rhs, (0, 10.0), r0, method="DOP853", rtol=1e-12, atol=1e-13,
                                events=[_skip_start(e) for e in ev], args=(sig,))
                end = sol.y[:, -1]
            assert np.max(np.abs(end - L[key][s])) < 5e-9, (s, sig, end, L[key][s])


def _skip_start(e):
    """Box-exit event that ignores the start point on the bottom face."""

    def f(t, r, sg):
        v = e(t, r, sg)
        return v if t > 1e-9 else (1.0 if v == 0 else v)

    f.terminal = True
    f.direction = 0
    return f


# --------------------------------------------------------------------------------------
# per-line failure handling
# --------------------------------------------------------------------------------------


def test_status_paths(orc):
    g = cubic_grid(9, 9, 9)
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    seeds = np.array([[1.5, 0.5, 0.5], [0.5, 0.5, 0.5]])
    L = orc.trace(B, g, seeds)
    assert L["status"][0] & orc.ORC_OUTSIDE
    assert np.isnan(L["tw"][0])
    assert L["status"][1] == 0
    # a planted NaN on the path
    Bn = B.copy()
    Bn[2, 6, 4, 4] = np.nan
    L = orc.trace(Bn, g, np.array([[0.5, 0.5, 0.1]]))
    assert L["status"][0] & orc.ORC_NONFINITE
    # a null region
    Bz = B.copy()
    Bz[:, 5:, :, :] = 0.0
    L = orc.trace(Bz, g, np.array([[0.5, 0.5, 0.1]]))
    assert L["status"][0] & orc.ORC_NULLB
    # step budget
    L = orc.trace(B, g, np.array([[0.5, 0.5, 0.1]]), opts={"max_steps": 1})
    assert L["status"][0] & orc.ORC_MAXSTEPS


def test_mixed_face_stencil(orc):
    """Neighbours ending on different faces (Section 2.1, the NaN case of Code2016):
    one-sided where one neighbour matches, NaN where none does; an end on a box
    edge is flagged."""
    g = cubic_grid(9, 9, 9)
    B = linear_field(g, np.zeros((3, 3)), [0.5, 0, 1.0])  # x1 < 0.5 -> top, x1 > 0.5 -> x+
    pl = Plane((0.485, 0.5, 0.0), (1, 0, 0), (0, 1, 0), 3, 3, 0.01, 0.01)
    r = orc.q2d(B, g, pl)
    L = r["lines"]
    assert list(L["face_f"][3:6]) == [5, 5, 1]
    st = r["status"]
    assert st[1, 1] & orc.ORC_ONESIDED and not st[1, 1] & orc.ORC_MIXEDFACE
    assert abs(r["q"][1, 1] - 2.0) < 1e-9  # one-sided with the top-ending neighbour
    assert st[1, 2] & orc.ORC_MIXEDFACE  # its only x neighbour ends on the top face
    pl2 = Plane((0.495, 0.5, 0.0), (1, 0, 0), (0, 1, 0), 2, 3, 0.01, 0.01)
    r2 = orc.q2d(B, g, pl2)
    assert np.all(r2["status"] & orc.ORC_MIXEDFACE)
    assert np.all(np.isnan(r2["q"]))
    # a line that lands on the x+/z+ edge
    L = orc.trace(B, g, np.array([[0.5, 0.5, 0.0]]))
    assert L["status"][0] & orc.ORC_EDGE


def test_q_at_least_two(orc):
    """Q >= 2, the theoretical minimum (Section 1): ||D||^2 >= 2 |det D| and, with
    flux conserved exactly, |det D| = |Bn1/Bn2|, so only the O(delta^2) error of the
    differences remains."""
    g = cubic_grid(9, 9, 9)
    B = _multilinear_solenoidal(g)
    r = orc.q2d(B, g, synth.plane_z0(32), {"tol": 1e-11})
    m = r["status"] == 0
    assert m.sum() > 0.5 * m.size
    assert np.nanmin(r["q"][m]) > 2 - 1e-4
    assert np.nanmax(r["q"][m]) > 2.5


def test_sampled_points_equal_full_map(orc):
    """The sampled-point entry points assemble Q exactly as the full maps do."""
    w = synth.config_c1(2, nseed=40)
    full = orc.q2d(w.field, w.grid, w.plane)
    rng = np.random.default_rng(0)
    pts = rng.choice(40 * 40, 60, replace=False)
    pts = np.concatenate([pts, [0, 39, 40 * 39]])  # map corners too
    sub = orc.q2d_points(w.field, w.grid, w.plane, pts)
    assert np.array_equal(sub["status"], full["status"].ravel()[pts])
    assert np.array_equal(np.isnan(sub["q"]), np.isnan(full["q"].ravel()[pts]))
    m = ~np.isnan(sub["q"])
    assert np.array_equal(sub["q"][m], full["q"].ravel()[pts][m])
    assert np.array_equal(sub["tw"], full["tw"].ravel()[pts])
    rng = np.random.default_rng(2)
    g = cubic_grid(17, 17, 13)
    pos, q = synth.draw_charges(rng, 5)
    B = synth.charges_field(g, pos, q)
    ux, uy, uz = g.upper
    vx = Voxels((ux / 16, uy / 16, uz / 12), (ux / 8, uy / 8, uz / 6), (8, 8, 6))
    f3 = orc.q3d(B, g, vx)
    pts = rng.choice(8 * 8 * 6, 50, replace=False)
    s3 = orc.q3d_points(B, g, vx, pts)
    assert np.array_equal(s3["status"], f3["status"].ravel()[pts])
    m = ~np.isnan(s3["q"])
    assert np.array_equal(s3["q"][m], f3["q"].ravel()[pts][m])


# --------------------------------------------------------------------------------------
# landing at grazing incidence: a polarity inversion line on the seed face
# --------------------------------------------------------------------------------------


def _arcade(g, x0):
    """B = (1, 0, -(x - x0)): arcades over the polarity inversion line x = x0 of the
    bottom face. A line from (x1, y1, 0) is the parabola z = ((x1-x0)^2 - (x-x0)^2)/2
    and comes back to z = 0 at x2 = 2 x0 - x1, y2 = y1, where Bn = x1 - x0 = -Bn0
    (Eq. rb)."""
    return linear_field(g, [[0, 0, 0], [0, 0, 0], [-1, 0, 0]], [1.0, 0.0, x0])


@pytest.mark.parametrize("dist", [1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8])
def test_pil_arcade_q_is_two(orc, dist):
    """Seeds on both sides of a polarity inversion line of the bottom face. The
    zero-length half is S1 (the seed), so both sides map seed -> far footpoint by
    x2 = 2 x0 - x1: a linear map with |Bn2/Bn0| = 1, hence Q = 2 exactly
    (Section 1, Eq. Q+-; Q >= 2). The far footpoint is met at the angle of the seed,
    which is |x1 - x0| at most: an end that is not converged on the crossing itself
    (rather than on the height above the face) moves Bn2, so Q, by a relative
    error/dist. Both ends must sit on the closed form."""
    g = cubic_grid(17, 17, 17)
    x0 = 0.5 + 1e-4 * math.pi
    B = _arcade(g, x0)
    d = 7e-4  # stencil spacing: neighbours stay off the inversion line
    for sgn in (-1.0, 1.0):
        xc = x0 + sgn * dist
        pl = Plane((xc - d, 0.5 - d, 0.0), (1, 0, 0), (0, 1, 0), 3, 3, d, d)
        r = orc.q2d(B, g, pl)
        assert r["status"][1, 1] == 0
        assert abs(r["q"][1, 1] - 2.0) < 1e-9, (sgn * dist, r["q"][1, 1])
        L = r["lines"]
        seeds = pl.points()
        far = np.where((L["face_f"] == 4)[:, None] & (np.abs(L["end_f"] - seeds).sum(1) > 0)[:, None],
                       L["end_f"], L["end_b"])
        assert np.max(np.abs(far[:, 0] - (2 * x0 - seeds[:, 0]))) < 1e-13
        assert np.max(np.abs(far[:, 1] - seeds[:, 1])) < 1e-14


def test_pil_arcade_map_straddling_the_pil(orc):
    """A 40 x 3 map across the inversion line with one seed 1e-9 from it: every point
    with central differences has Q = 2 to rounding (none drops below 2 - O(delta^2))."""
    g = cubic_grid(17, 17, 17)
    x0 = 0.5 + 1e-4 * math.pi
    B = _arcade(g, x0)
    d = 1.37e-3
    n = 40
    ox = x0 + 1e-9 - 20 * d
    pl = Plane((ox, 0.5 - d, 0.0), (1, 0, 0), (0, 1, 0), n, 3, d, d)
    r = orc.q2d(B, g, pl)
    q = r["q"][1, 1:-1]
    st = r["status"][1, 1:-1]
    assert np.all(st == 0)
    assert np.max(np.abs(q - 2.0)) < 1e-8, np.max(np.abs(q - 2.0))


# --------------------------------------------------------------------------------------
# 3-D maps: rotated S0 (Section 4) and B . grad Q = 0 (Section 1, Eq. qline)
# --------------------------------------------------------------------------------------


def _sheared_oblique(g, s, y0, by=0.3):
    """B = (1, by, s (y - y0)): y = y1 + by (x - x1) and z picks up
    s (y1 - y0)(x - x1) + s by (x - x1)^2 / 2, so between the faces x = 0 and x = 1
    (S1, S2 with Bn = Bx = 1) the map is (y, z) -> (y + by, z + s (y - y0) + s by / 2):
    Jacobian [[1, 0], [s, 1]] and Q = 2 + s^2 (Section 1, Eq. Q+-)."""
    return linear_field(g, [[0, 0, 0], [0, 0, 0], [0, s, 0]], [1.0, by, -s * y0])


def test_rotated_s0_closed_form(orc):
    """Voxels of a 3-D map where |Bz/B| < 0.05 take S0 perpendicular to B with four
    extra lines (Section 4); elsewhere S0 is the voxel's z plane. Q is a property of
    the line (Eq. qline), so both must give 2 + s^2. A voxel with Bz = 0 has no
    usable z-plane stencil at all: only the rotated S0 gives Q there."""
    g = cubic_grid(17, 17, 17)
    s, y0 = 0.5, 0.4
    B = _sheared_oblique(g, s, y0)
    dv = 1e-4
    opts = {"tol": 1e-12}
    seen_rot = seen_plain = 0
    for yc in (y0, y0 + 0.003, y0 - 0.02, y0 + 0.08, y0 - 0.12, y0 + 0.2):
        vx = Voxels((0.45 - dv, yc - dv, 0.5), (dv, dv, 0.01), (3, 3, 1))
        r = orc.q3d(B, g, vx, opts)
        q, st = r["q"][0, 1, 1], r["status"][0, 1, 1]
        rot = abs(s * (yc - y0)) < 0.05 * math.sqrt(1 + 0.09 + (s * (yc - y0)) ** 2)
        assert bool(st & orc.ORC_ROTATED) == rot, (yc, st)
        assert (int(st) & ~orc.ORC_ROTATED) == 0, (yc, st)
        assert abs(q - (2 + s * s)) < 1e-6, (yc, q)
        seen_rot += rot
        seen_plain += not rot
    assert seen_rot >= 3 and seen_plain >= 2


def _interp_div(B, g, r):
    """Trilinear B and the divergence of the trilinear interpolant at r (numpy; the
    cell's corner values weighted by Eq. interp / w0 / w1 and by their derivatives)."""
    n = (g.nx, g.ny, g.nz)
    c, t = [], []
    for a in range(3):
        x = (r[a] - g.origin[a]) / g.spacing[a]
        i = min(max(int(math.floor(x)), 0), n[a] - 2)
        c.append(i)
        t.append(x - i)
    i, j, k = c
    cube = B[:, k:k + 2, j:j + 2, i:i + 2]
    wx, wy, wz = (np.array([1 - t[0], t[0]]), np.array([1 - t[1], t[1]]),
                  np.array([1 - t[2], t[2]]))
    d = np.array([-1.0, 1.0])
    val = np.einsum("czyx,z,y,x->c", cube, wz, wy, wx)
    div = (np.einsum("zyx,z,y,x->", cube[0], wz, wy, d) / g.spacing[0] +
           np.einsum("zyx,z,y,x->", cube[1], wz, d, wx) / g.spacing[1] +
           np.einsum("zyx,z,y,x->", cube[2], d, wy, wx) / g.spacing[2])
    return val, div


def _div_integral(B, g, p0, z_end):
    """Integral of div(B)/|B| ds along the line from p0 (following B) up to the plane
    z = z_end, by scipy's DOP853 on the trilinear interpolant (independent of the
    oracle's integrator)."""
    from scipy.integrate import solve_ivp

    def rhs(s, y):
        b, dv = _interp_div(B, g, y[:3])
        bm = np.linalg.norm(b)
        return np.concatenate([b / bm, [dv / bm]])

    def hit(s, y):
        return y[2] - z_end

    hit.terminal = True
    sol = solve_ivp(rhs, (0.0, 5.0), np.concatenate([p0, [0.0]]), method="DOP853",
                    rtol=1e-11, atol=1e-13, events=hit)
    assert sol.status == 1
    return sol.y[3, -1], sol.y[:3, -1]


def _line_lattice(p0, p1, z0, z1, step):
    """A voxel lattice of two layers (z0, z1) with a voxel centre on p0 and one on p1
    (p1 - p0 is a whole number of x and y spacings near `step`); returns the voxels
    and the flat indices of the two centres."""
    dx, dy = p1[0] - p0[0], p1[1] - p0[1]
    mx_, my_ = max(1, int(round(abs(dx) / step))), max(1, int(round(abs(dy) / step)))
    sx, sy = abs(dx) / mx_, abs(dy) / my_
    lo = np.minimum(p0, p1)
    origin = (lo[0] - sx, lo[1] - sy, z0)
    nx_, ny_ = mx_ + 3, my_ + 3
    vx = Voxels(origin, (sx, sy, z1 - z0), (nx_, ny_, 2))
    i0, j0 = int(round((p0[0] - origin[0]) / sx)), int(round((p0[1] - origin[1]) / sy))
    i1, j1 = int(round((p1[0] - origin[0]) / sx)), int(round((p1[1] - origin[1]) / sy))
    a, b = j0 * nx_ + i0, (ny_ + j1) * nx_ + i1
    pts = vx.points()
    assert np.max(np.abs(pts[a] - p0)) < 1e-12 and np.max(np.abs(pts[b] - p1)) < 1e-12
    return vx, a, b


def _lines_through_two_layers(orc, B, g, k0, k1, candidates, opts):
    """Seeds p0 on the plane half a cell above node plane k0 whose forward lines rise
    through node plane k1, and their crossing points p1 there: the same line traced
    in the sub-box below plane k1 (trilinear interpolation is local to a cell, so
    the sub-box holds the same interpolated field) ends on p1."""
    z0, z1 = g.spacing[2] * (k0 + 0.5), g.spacing[2] * k1
    gs = synth.Grid(g.nx, g.ny, k1 + 1, g.origin, g.spacing)
    sub = np.ascontiguousarray(B[:, : k1 + 1])
    out = []
    for (x, y) in candidates:
        p0 = np.array([x, y, z0])
        L = orc.trace(sub, gs, p0[None, :], opts=opts)
        if L["face_f"][0] == 5:
            out.append((p0, L["end_f"][0]))
    return z0, z1, out


def test_p9_voxels_on_one_line_share_tw_length_and_q(orc):
    """B . grad Q = 0 (Section 1, Eq. qline) on a 3-D map whose voxel lattice puts
    two voxels of different layers on one field line. They must get the same Tw and
    length (one line). Their Q comes from Method I through two different S0 planes
    with |det D| replaced by the normal-field ratio (Eq. D+-3, Eq. Bn1), which
    assumes that flux is conserved along the line. The trilinear interpolant of a
    divergence-free field is not exactly divergence-free, and flux along a thin
    tube grows as exp(int div B / |B| ds), so the two values must differ by exactly
    Q(p0) / Q(p1) = exp(2 int_{p0}^{p1} div B / |B| ds) (up to the O(delta^2) error
    of the differences); the integral is computed independently with scipy."""
    bad = orc.FATAL | orc.ORC_MIXEDFACE | orc.ORC_EDGE | orc.ORC_ONESIDED
    rng = np.random.default_rng(11)
    g = cubic_grid(33, 33, 33)
    pos, qq = synth.draw_charges(rng, 4)
    B = synth.charges_field(g, pos, qq)
    opts = {"tol": 1e-12}
    z0, z1, pairs = _lines_through_two_layers(
        orc, B, g, 8, 12, ((0.41, 0.47), (0.36, 0.61), (0.62, 0.58)), opts)
    assert len(pairs) >= 2
    checked = 0
    for p0, p1 in pairs:
        I, end = _div_integral(B, g, p0, z1)
        assert np.max(np.abs(end - p1)) < 1e-8  # the same line
        # the full-map entry point on a coarse lattice (delta ~ 2e-3)
        vx, a, b = _line_lattice(p0, p1, z0, z1, 2e-3)
        r = orc.q3d(B, g, vx, opts)
        q, tw, ln, st = (r[k].ravel() for k in ("q", "tw", "len", "status"))
        if (st[a] | st[b]) & bad:
            continue
        assert abs(tw[a] - tw[b]) < 1e-9 and abs(ln[a] - ln[b]) < 1e-9
        assert abs(math.log(q[a] / q[b]) - 2 * I) < 1.5e-3
        m = (st & bad) == 0
        assert np.nanmin(q[m]) > 2 - 1e-3  # Q >= 2 - O(delta^2)
        # sampled points on a fine lattice (delta ~ 2.5e-4): the O(delta^2) part shrinks
        vx, a, b = _line_lattice(p0, p1, z0, z1, 2.5e-4)
        r = orc.q3d_points(B, g, vx, np.array([a, b]), opts)
        assert not (r["status"] & bad).any()
        assert abs(math.log(r["q"][0] / r["q"][1]) - 2 * I) < 3e-5, (r["q"], I)
        checked += 1
    assert checked >= 2


def test_p9_solenoidal_interpolant_q_is_a_line_invariant(orc):
    """With a field whose trilinear interpolant is exactly divergence-free, Method I
    through any S0 on the line gives one Q: voxels of two layers on one line agree
    to the O(delta^2) error of the differences (Section 1, Eq. qline)."""
    bad = orc.FATAL | orc.ORC_MIXEDFACE | orc.ORC_EDGE | orc.ORC_ONESIDED
    g = cubic_grid(9, 9, 9)
    B = _multilinear_solenoidal(g)
    opts = {"tol": 1e-12}
    z0, z1, pairs = _lines_through_two_layers(
        orc, B, g, 2, 5, ((0.47, 0.52), (0.3, 0.6), (0.6, 0.35)), opts)
    assert len(pairs) >= 2
    for p0, p1 in pairs:
        vx, a, b = _line_lattice(p0, p1, z0, z1, 1e-3)
        r = orc.q3d(B, g, vx, opts)
        q, tw, ln, st = (r[k].ravel() for k in ("q", "tw", "len", "status"))
        assert not ((st[a] | st[b]) & bad)
        assert abs(tw[a] - tw[b]) < 1e-10 and abs(ln[a] - ln[b]) < 1e-10
        assert abs(q[a] / q[b] - 1) < 1e-5, (q[a], q[b])
        assert q[a] > 2.05  # a non-trivial map


# --------------------------------------------------------------------------------------
# Method II (Section 2.1, Eq. rb2, Eq. q_scott): Q and Q_perp from tangent vectors
# --------------------------------------------------------------------------------------


@pytest.mark.parametrize("way", [1, 2])
def test_m2_uniform_and_tilted_fields(orc, way):
    """Uniform B: Q = Q_perp = 2. Tilted uniform B = (bx, 0, bz) from the bottom to
    the side face x+: Q = r + 1/r with r = bz/bx (the projection effect of S1, S2 on
    the faces), while Q_perp = 2: planes perpendicular to B remove it (Section 2.1)."""
    g = cubic_grid(17, 17, 17)
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    r = orc.method2(B, g, np.array([[0.3, 0.4, 0.0], [0.5, 0.5, 0.5]]), way)
    assert np.all(r["status"] == 0)
    assert np.allclose(r["q"], 2.0, atol=1e-12) and np.allclose(r["qperp"], 2.0, atol=1e-12)
    bx, bz = 2.0, 1.0
    B = linear_field(g, np.zeros((3, 3)), [bx, 0, bz])
    r = orc.method2(B, g, np.array([[0.7, 0.5, 0.0], [0.8, 0.3, 0.0]]), way)
    assert np.all(r["lines"]["face_f"] == 1)
    assert np.allclose(r["q"], bz / bx + bx / bz, rtol=1e-10)
    assert np.allclose(r["qperp"], 2.0, rtol=1e-10)


def test_m2_sheared_field(orc):
    """B = (s (y - y0), 0, 1): the lines are straight, x2 = x1 + s (y1 - y0) L, so
    Q = 2 + s^2 L^2 with S1, S2 on the faces; along a line U and V stay
    perpendicular to B with dV/ds = s / (1 + a^2) e1 (a = s (y1 - y0), e1 the
    in-plane unit vector perpendicular to B), which gives
    Q_perp = 2 + s^2 L^2 / (1 + a^2) (Eq. rb2, Eq. q_scott). Way 2 differentiates
    the exact interpolant (to its 1e-3-cell offsets); way 1's node differences of
    B/B converge at second order in the grid spacing."""
    s, y0 = 0.5, 0.5
    ys = np.array([0.3, 0.5, 0.7])
    seeds = np.c_[np.full(3, 0.45), ys, np.zeros(3)]
    a = s * (ys - y0)
    q_exp = 2 + s * s
    qp_exp = 2 + s * s / (1 + a * a)
    errs = []
    for n in (17, 33):
        g = cubic_grid(n, n, n)
        B = linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1])
        r2 = orc.method2(B, g, seeds, 2)
        assert np.allclose(r2["q"], q_exp, rtol=1e-8)
        assert np.allclose(r2["qperp"], qp_exp, rtol=1e-8)
        r1 = orc.method2(B, g, seeds, 1)
        errs.append(max(np.abs(r1["q"] / q_exp - 1).max(), np.abs(r1["qperp"] / qp_exp - 1).max()))
    assert errs[1] < 2e-4 and 3.0 < errs[0] / errs[1] < 5.0, errs


def test_m2_hyperbolic_field(orc):
    """B = (k(x - xc), -k(y - yc), 1): Q = 2 cosh(2 kL) (Eq. Q+-, Eq. q_scott); way 1
    converges to it at second order in the grid spacing."""
    kL = 2.0
    seeds = np.array([[0.5 + 0.05 * math.exp(-kL), 0.52, 0.0]])
    q_exp = 2 * math.cosh(2 * kL)
    errs = []
    for n in (17, 33, 65):
        g = cubic_grid(n, n, n)
        B = linear_field(g, [[kL, 0, 0], [0, -kL, 0], [0, 0, 0]], [-kL * 0.5, kL * 0.5, 1])
        r = orc.method2(B, g, seeds, 2)
        assert abs(r["q"][0] / q_exp - 1) < 1e-7
        errs.append(abs(orc.method2(B, g, seeds, 1)["q"][0] / q_exp - 1))
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def test_m2_agrees_with_method1_at_the_same_seeds(orc):
    """Both methods give the Q of one map (Eq. q_scott is equivalent to Eq. Q+-,
    Section 2.1). At seeds on the bottom face Method I's S0 (the face) and Method II's
    (perpendicular to B) pass through the same point, so the flux substitution
    treats them alike, and Method II with offset differences matches Method I's
    differences over delta = 1e-4 to their O(delta^2) and O(offset^2) errors. The
    results do not depend on the sign of B."""
    rng = np.random.default_rng(7)
    g = cubic_grid(33, 33, 33)
    pos, qq = synth.draw_charges(rng, 4)
    B = synth.charges_field(g, pos, qq)
    d = 1e-4
    pts = np.c_[np.random.default_rng(1).uniform(0.2, 0.8, (30, 2)), np.zeros(30)]
    qi = []
    for p in pts:
        r = orc.q2d(B, g, _plane(p, d), {"tol": 1e-12})
        qi.append(r["q"][1, 1] if r["status"][1, 1] == 0 else np.nan)
    qi = np.array(qi)
    r2 = orc.method2(B, g, pts, 2, {"tol": 1e-12})
    ok = np.isfinite(qi) & (r2["status"] == 0) & (qi < 1e3)
    assert ok.sum() >= 25 and np.nanmax(qi[ok]) > 10
    assert np.max(np.abs(r2["q"][ok] / qi[ok] - 1)) < 1e-3
    rn = orc.method2(-B, g, pts, 2, {"tol": 1e-12})
    assert np.allclose(rn["q"][ok], r2["q"][ok], rtol=1e-8)
    assert np.allclose(rn["qperp"][ok], r2["qperp"][ok], rtol=1e-8)


# --------------------------------------------------------------------------------------
# stretched rectilinear grids (Section 2.2: nodes x_i, y_j, z_k, cell by bisection;
# Eq. interp / w0 / w1 with the cell's own widths)
# --------------------------------------------------------------------------------------


def _stretched(nx, ny, nz, seed=5, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Strictly increasing random node coordinates: cell widths drawn in [0.3, 1.7]
    times the mean, so neighbouring cells differ by up to a factor of five."""
    rng = np.random.default_rng(seed)
    ax = []
    for n, a, b in zip((nx, ny, nz), lo, hi):
        w = rng.uniform(0.3, 1.7, n - 1)
        x = np.concatenate([[0.0], np.cumsum(w)])
        x = a + (b - a) * x / x[-1]
        x[-1] = b
        ax.append(x)
    return synth.stretched_grid(*ax)


def test_stretched_curl_exact_for_quadratic_field(orc):
    """On unequal spacings the three-node difference is the derivative of the
    quadratic through the nodes: exact for quadratic fields at every node, the
    boundary ones included (a wrong weight or a uniform-spacing formula fails)."""
    g = _stretched(7, 8, 9, lo=(0.1, -0.2, 0.3), hi=(1.6, 1.2, 1.5))
    x, y, z = g.axes()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    B = np.stack([X * Y + 2 * Z * Z - Y, Y * Z - 3 * X * X + X * Z, X * Y * 0.5 + Z * X - Y * Y])
    J = np.stack([(0.5 * X - 2 * Y) - (Y + X), 4 * Z - (0.5 * Y + Z), (-6 * X + Z) - (X - 1)])
    assert np.max(np.abs(orc.curl(B, g) - J)) < 1e-10


def test_stretched_interp_matches_scipy_trilinear(orc):
    """Eq. interp / w0 / w1 with each cell's own node coordinates, against scipy's
    linear RegularGridInterpolator on the same rectilinear grid."""
    from scipy.interpolate import RegularGridInterpolator

    rng = np.random.default_rng(3)
    g = _stretched(6, 5, 7, lo=(0.0, 1.0, -1.0), hi=(1.5, 3.0, 0.2))
    B = rng.standard_normal((3,) + g.shape)
    x, y, z = g.axes()
    pts = np.stack([rng.uniform(x[0], x[-1], 60), rng.uniform(y[0], y[-1], 60),
                    rng.uniform(z[0], z[-1], 60)], axis=1)
    for c in range(3):
        f = RegularGridInterpolator((x, y, z), np.transpose(B[c], (2, 1, 0)), method="linear")
        ref = f(pts)
        for p, r in zip(pts, ref):
            cell = [min(int(np.searchsorted(ax, p[a], side="right")) - 1, ax.size - 2)
                    for a, ax in enumerate((x, y, z))]
            assert abs(orc.interp(B, g, cell, p)[c] - r) < 1e-12


def test_stretched_linear_fields_closed_forms(orc):
    """A field linear in x, y, z is its own trilinear interpolant on any rectilinear
    grid, and its curl is exact: the closed forms of P1, P3, P4 and P5 hold on a
    grid whose neighbouring cells differ by up to five times in width. They then
    bound the cell lookup, the landings on faces at unequal positions and the
    error norm in each cell's widths."""
    g = _stretched(13, 12, 15, seed=7)
    # P1: identity map, Q = 2, length Lz
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    pl = synth.plane_z0(12)
    r = orc.q2d(B, g, pl)
    assert np.all(r["status"] & orc.FATAL == 0)
    assert np.allclose(r["q"], 2.0, atol=1e-10)
    assert np.allclose(r["len"], 1.0, atol=1e-12)
    assert np.allclose(r["lines"]["end_f"][:, :2], pl.points()[:, :2], atol=1e-12)
    # P3: sheared field, Q = 2 + s^2, Tw = -s / (4 pi sqrt(1 + s^2 (y1 - y0)^2))
    s, y0 = 0.5, 0.5
    B = linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1])
    pl = _plane((0.45, 0.3, 0.0), 0.01, n=5)
    r = orc.q2d(B, g, pl)
    seeds = pl.points()
    y1 = seeds[:, 1]
    assert np.allclose(r["q"], 2 + s * s, rtol=1e-9)
    assert np.allclose(r["tw"].ravel(), -s / (4 * np.pi * np.sqrt(1 + s * s * (y1 - y0) ** 2)),
                       atol=1e-11)
    assert np.allclose(r["lines"]["end_f"][:, 0], seeds[:, 0] + s * (y1 - y0), atol=1e-11)
    # P4: hyperbolic field, Q = 2 cosh 2kL
    kL = 3.0
    xc = yc = 0.5
    B = linear_field(g, [[kL, 0, 0], [0, -kL, 0], [0, 0, 0]], [-kL * xc, kL * yc, 1])
    pl = _plane((xc + 0.2 * math.exp(-kL), yc + 0.1, 0.0), 1e-4, n=3)
    r = orc.q2d(B, g, pl)
    assert np.all(r["lines"]["face_f"] == 5)
    assert abs(r["q"][1, 1] / (2 * math.cosh(2 * kL)) - 1) < 1e-6
    # P5: twisted field, Tw = qL / (2 pi sqrt(1 + q^2 rho^2)), Q = 2
    q = 2 * math.pi
    B0 = 0.7
    B = linear_field(g, [[0, -q * B0, 0], [q * B0, 0, 0], [0, 0, 0]], [q * B0 * yc, -q * B0 * xc, B0])
    pl = _plane((xc + 0.05, yc, 0.0), 0.002, n=3)
    r = orc.q2d(B, g, pl)
    rho = np.hypot(pl.points()[:, 0] - xc, pl.points()[:, 1] - yc)
    assert np.allclose(r["tw"].ravel(), q / (2 * np.pi * np.sqrt(1 + q * q * rho * rho)), atol=1e-9)
    assert abs(r["q"][1, 1] - 2.0) < 1e-6


def test_stretched_seeds_on_nodes_and_faces(orc):
    """Seeds exactly on interior node planes and on the top face of a stretched
    grid: bisection puts a point on node x_i into cell i (the last cell for the last
    node), so lines start in the right cell and end where the uniform field sends
    them, with the length of the box above the seed."""
    g = _stretched(9, 9, 11, seed=11)
    x, y, z = g.axes()
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    seeds = np.array([[x[3], y[4], z[2]], [x[0], y[8], z[5]], [x[8], y[0], z[10]],
                      [0.5 * (x[1] + x[2]), y[7], z[9]]])
    r = orc.trace(B, g, seeds)
    # seeds 1 and 2 lie on box faces, so their lines run along box edges (EDGE bit)
    assert np.all((r["status"] & orc.FATAL) == 0)
    assert np.allclose(r["end_f"][:, :2], seeds[:, :2], atol=1e-14)
    assert np.allclose(r["end_f"][:, 2], z[-1], atol=0) and np.allclose(r["end_b"][:, 2], z[0], atol=0)
    assert np.allclose(r["len"], z[-1] - z[0], atol=1e-12)


def test_stretched_with_uniform_nodes_equals_uniform(orc, charge_cube):
    """A grid whose node coordinates are given explicitly but are uniform is the
    uniform grid: the stretched code paths give the uniform ones' map (Q, Tw,
    footpoints) to within the integrators' tolerance."""
    g, B = charge_cube
    gs = synth.stretched_grid(*g.axes())
    pl = _plane((0.4, 0.55, 0.0), 0.01, n=6)
    ru = orc.q2d(B, g, pl)
    rs = orc.q2d(B, gs, pl)
    m = (ru["status"] & orc.FATAL) == 0
    assert m.all() and np.array_equal(ru["status"], rs["status"])
    assert np.allclose(rs["q"], ru["q"], rtol=1e-7)
    assert np.allclose(rs["tw"], ru["tw"], atol=1e-9)
    for k in ("end_b", "end_f"):
        assert np.allclose(rs["lines"][k], ru["lines"][k], atol=1e-9)


# --------------------------------------------------------------------------------------
# Method I with S1, S2 perpendicular to B (Q_perp, Section 2.1) and the length edge map
# --------------------------------------------------------------------------------------


def test_perp_uniform_and_tilted_fields(orc):
    """Uniform field: Q_perp = 2 and no length edge. Tilted uniform field ending on the
    side face x+: Q = r + 1/r there (the projection effect of the face, Section 2.1)
    but Q_perp = 2, and the length (1 - x1) |B| / bx changes at |B| / bx per unit x1."""
    g = cubic_grid(11, 11, 11)
    B = linear_field(g, np.zeros((3, 3)), [0, 0, 1])
    r = orc.q2d_perp(B, g, synth.plane_z0(8))
    assert np.allclose(r["qperp"], 2.0, atol=1e-12) and np.allclose(r["fledge"], 0.0, atol=1e-12)
    bx, bz = 2.0, 1.0
    B = linear_field(g, np.zeros((3, 3)), [bx, 0, bz])
    pl = synth.plane_z0(20)
    r = orc.q2d_perp(B, g, pl)
    o = orc.q2d(B, g, pl)
    side = (o["lines"]["face_f"] == 1).reshape(20, 20)
    inner = side & ((r["status"] & (orc.ORC_ONESIDED | orc.ORC_MIXEDFACE)) == 0)
    assert inner.sum() > 20
    assert np.allclose(o["q"][inner], bz / bx + bx / bz, rtol=1e-9)
    assert np.allclose(r["qperp"][inner], 2.0, rtol=1e-9)
    assert np.allclose(r["fledge"][inner], math.hypot(bx, bz) / bx, rtol=1e-9)


def test_perp_sheared_field(orc):
    """B = (s(y - y0), 0, 1): Q_perp = 2 + s^2 / (1 + a^2), a = s(y1 - y0) (the closed
    form Method II gives too), and the length sqrt(1 + a^2) has |grad| =
    s |a| / sqrt(1 + a^2) (central differences inside the seed grid)."""
    g = cubic_grid(11, 11, 11)
    s, y0 = 0.5, 0.5
    B = linear_field(g, [[0, s, 0], [0, 0, 0], [0, 0, 0]], [-s * y0, 0, 1])
    pl = _plane((0.45, 0.27, 0.0), 0.01, n=5)
    r = orc.q2d_perp(B, g, pl)
    a = (s * (pl.points()[:, 1] - y0)).reshape(5, 5)
    assert np.allclose(r["qperp"], 2 + s * s / (1 + a * a), rtol=1e-10)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(r["fledge"][inner], (np.abs(s * a) / np.sqrt(1 + a * a))[inner], atol=1e-6)


def test_perp_agrees_with_method2(orc):
    """On the 4-charge cube Method I's Q_perp (neighbour differences, d = 1e-4) and
    Method II's (tangent vectors) agree to the stencil's O(d^2) error: two
    independent ways to the same Q_perp."""
    w = synth.config_c1(0)
    for centre in ((0.37, 0.52), (0.61, 0.44), (0.5, 0.3)):
        pl = _plane((centre[0], centre[1], 0.0), 1e-4, n=3)
        r = orc.q2d_perp(w.field, w.grid, pl, {"tol": 1e-12})
        m = orc.method2(w.field, w.grid, pl.points()[4:5], 2, {"tol": 1e-12})
        assert abs(r["qperp"][1, 1] / m["qperp"][0] - 1) < 1e-4, (centre, r["qperp"][1, 1], m["qperp"][0])


# --------------------------------------------------------------------------------------
# a cylindrical mapping surface (Section 3: B = (x, -y, 0) with S1, S2 on x^2 + y^2 = 1)
# --------------------------------------------------------------------------------------


def _cyl_box():
    return synth.Grid(31, 31, 11, (-1.5, -1.5, 0.0), (0.1, 0.1, 0.1))


def test_cylinder_paper_example(orc):
    """B = (x, -y, 0), mapping surface x^2 + y^2 = 1: for 0 < theta < pi/2 the line
    inside the cylinder maps theta1 -> pi/2 - theta1 at the same z, so Q = 2
    (Section 3); Tw = 0 (curl-free); the length is the arc of the hyperbola
    x y = sin(2 theta1) / 2 between the two crossings (integrated here by scipy);
    the half pointing out of the cylinder ends at its seed."""
    from scipy.integrate import quad

    g = _cyl_box()
    B = linear_field(g, [[1, 0, 0], [0, -1, 0], [0, 0, 0]], [0, 0, 0])
    cyl = synth.Cylinder((0.0, 0.0), 1.0, 0.1, 0.05, 27, 0.2, 0.1, 5)
    r = orc.qcyl(B, g, cyl, {"tol": 1e-10})
    th = cyl.theta0 + cyl.dtheta * np.arange(cyl.ntheta)
    inner = (slice(1, -1), slice(1, -1))
    assert np.all(r["status"][inner] == 0)
    assert np.allclose(r["q"][inner], 2.0, rtol=1e-9)
    assert np.allclose(r["tw"], 0.0, atol=1e-12)
    L = r["lines"]
    fb = L["face_b"].reshape(cyl.nz, cyl.ntheta)
    ff = L["face_f"].reshape(cyl.nz, cyl.ntheta)
    assert np.all(fb == orc.ORC_FACE_CYL) and np.all(ff == orc.ORC_FACE_CYL)
    # B . n = cos 2 theta: below pi/4 the forward half leaves at once, above it the backward one
    eb = L["end_b"].reshape(cyl.nz, cyl.ntheta, 3)
    ef = L["end_f"].reshape(cyl.nz, cyl.ntheta, 3)
    seeds = cyl.points().reshape(cyl.nz, cyl.ntheta, 3)
    far = np.where((th < math.pi / 4)[None, :, None], eb, ef)
    near = np.where((th < math.pi / 4)[None, :, None], ef, eb)
    assert np.allclose(near, seeds, atol=0)
    assert np.allclose(np.arctan2(far[..., 1], far[..., 0]), math.pi / 2 - th[None, :], atol=1e-10)
    assert np.allclose(far[..., 2], seeds[..., 2], atol=1e-12)
    for k in (0, 5, 20):
        c = 0.5 * math.sin(2 * th[k])
        x1, x2 = sorted((math.cos(th[k]), math.sin(th[k])))
        arc = quad(lambda x: math.sqrt(1 + c * c / x ** 4), x1, x2, epsabs=1e-13)[0]
        assert abs(r["len"][2, k] - arc) < 1e-9


def test_cylinder_tilted_uniform_field(orc):
    """B = (1, 0, bz) through the cylinder: a line from theta1 (pi/2 < theta1 < 3pi/2,
    where B points inward) crosses to pi - theta1 and rises 2 bz |cos theta1|, so on
    (r theta, z) coordinates D = [[-1, 0], [2 bz sin theta1, 1]], |Bn1/Bn2| = 1 and
    Q = 2 + 4 bz^2 sin^2 theta1 (the central difference over theta1 +- dtheta gives
    that entry times sin(dtheta)/dtheta exactly); the length is 2 |cos theta1|
    sqrt(1 + bz^2). The seed row straddles theta = pi, where the arc-length
    coordinate wraps."""
    g = _cyl_box()
    bz = 0.3
    B = linear_field(g, np.zeros((3, 3)), [1.0, 0.0, bz])
    cyl = synth.Cylinder((0.0, 0.0), 1.0, 2.0, 0.04, 56, 0.1, 0.02, 4)
    r = orc.qcyl(B, g, cyl, {"tol": 1e-11})
    th = cyl.theta0 + cyl.dtheta * np.arange(cyl.ntheta)
    inner = (slice(1, -1), slice(1, -1))
    c = 2 * bz * np.sin(th) * math.sin(cyl.dtheta) / cyl.dtheta
    qexp = np.broadcast_to(2 + c * c, r["q"].shape)
    assert np.all(r["status"][inner] == 0)
    assert np.allclose(r["q"][inner], qexp[inner], rtol=1e-7)
    lexp = np.broadcast_to(2 * np.abs(np.cos(th)) * math.sqrt(1 + bz * bz), r["len"].shape)
    assert np.allclose(r["len"], lexp, atol=1e-10)


def test_cylinder_short_chords_near_tangency(orc):
    """B = (1, 0, 0) with seeds just past theta = pi/2, where B barely points into
    the cylinder: the chords to pi - theta1 are far shorter than a first step (2
    |cos theta1| down to 2e-6), so the far crossing is bracketed from the surface
    itself; ends and lengths as the closed form gives them. At a grazing angle a the
    crossing is conditioned by phi's rounding, about 1e-16 / (2 a) along the line."""
    g = _cyl_box()
    B = linear_field(g, np.zeros((3, 3)), [1.0, 0.0, 0.0])
    for d in (1e-2, 1e-4, 1e-6):
        cyl = synth.Cylinder((0.0, 0.0), 1.0, math.pi / 2 + d, d / 4, 3, 0.5, 0.1, 3)
        r = orc.qcyl(B, g, cyl, {"tol": 1e-12})
        th = cyl.theta0 + cyl.dtheta * np.arange(3)
        eb = r["lines"]["end_b"].reshape(3, 3, 3)
        ef = r["lines"]["end_f"].reshape(3, 3, 3)
        # B . n = cos theta < 0: the forward half runs inside, the backward one ends at once
        assert np.allclose(eb, cyl.points().reshape(3, 3, 3), atol=0)
        tol = 1e-13 + 4e-16 / d
        assert np.allclose(np.arctan2(ef[..., 1], ef[..., 0]), math.pi - th[None, :], rtol=0, atol=tol)
        assert np.allclose(r["len"], np.broadcast_to(2 * np.abs(np.cos(th)), (3, 3)), rtol=0, atol=2 * tol)
