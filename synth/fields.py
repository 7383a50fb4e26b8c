"""Seeded field cubes and seed grids.

Layout convention used everywhere in this repository: a field is a float array of
shape (3, nz, ny, nx) holding the Bx, By, Bz node planes, x fastest, so node
(i, j, k) of component c sits at flat offset ((k * ny + j) * nx + i) of plane c.
Nodes sit at x_i = origin_x + i * dx (likewise y, z): a uniform Cartesian grid,
the case the paper's trilinear interpolation (Section 2.2) is written for; or, on a
stretched axis, at the given node coordinates x_i (a stretched rectilinear grid,
which the paper's code also accepts).

Everything here is computed in float64 and cast once at the end; the cast array
*is* the field that both the oracle and the GPU path see.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np


# --------------------------------------------------------------------------------------
# grid and seed descriptors
# --------------------------------------------------------------------------------------


@dataclass
class Grid:
    """Node grid: n = (nx, ny, nz) nodes, node (i,j,k) at origin + (i,j,k)*spacing;
    an axis whose entry of `coords` is an array has its nodes there instead
    (strictly increasing, n values; origin and spacing then unused on that axis)."""

    nx: int
    ny: int
    nz: int
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    spacing: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    coords: Optional[Tuple[Optional[np.ndarray], Optional[np.ndarray], Optional[np.ndarray]]] = None

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def upper(self) -> Tuple[float, float, float]:
        return tuple(float(x[-1]) for x in self.axes())

    @property
    def lower(self) -> Tuple[float, float, float]:
        return tuple(float(x[0]) for x in self.axes())

    def coord(self, a: int) -> Optional[np.ndarray]:
        """Node coordinates of a stretched axis a, else None."""
        if self.coords is None or self.coords[a] is None:
            return None
        return np.ascontiguousarray(self.coords[a], dtype=np.float64)

    @property
    def stretched(self) -> bool:
        return any(self.coord(a) is not None for a in range(3))

    def axes(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        out = []
        for a, (o, n, d) in enumerate(zip(self.origin, (self.nx, self.ny, self.nz), self.spacing)):
            c = self.coord(a)
            out.append(c if c is not None else o + d * np.arange(n, dtype=np.float64))
        return tuple(out)


def cubic_grid(nx: int, ny: int, nz: int) -> Grid:
    """Cubic cells with spacing 1/(nx-1): the x extent is one box unit."""
    d = 1.0 / (nx - 1)
    return Grid(nx, ny, nz, (0.0, 0.0, 0.0), (d, d, d))


def geometric_axis(n: int, lo: float, hi: float, ratio: float) -> np.ndarray:
    """n nodes from lo to hi whose cell widths grow by `ratio` from one cell to the
    next (ratio 1: uniform)."""
    w = ratio ** np.arange(n - 1, dtype=np.float64)
    x = np.concatenate([[0.0], np.cumsum(w)])
    x = lo + (hi - lo) * x / x[-1]
    x[-1] = hi
    return x


def clustered_axis(n: int, lo: float, hi: float, centre: float, strength: float) -> np.ndarray:
    """n nodes from lo to hi, denser around `centre` (a sinh map of a uniform
    parameter; strength 0: uniform)."""
    t = np.linspace(-1.0, 1.0, n)
    if strength == 0:
        return lo + (hi - lo) * (t + 1) / 2
    c = (centre - lo) / (hi - lo) * 2 - 1
    # x(t) = c + sinh(strength (t - t0)) / sinh(strength) scaled so x(-1) = -1, x(1) = 1
    a = np.arcsinh((1 + c) * math.sinh(strength)) / strength
    b = np.arcsinh((1 - c) * math.sinh(strength)) / strength
    tt = -a + (t + 1) / 2 * (a + b)
    x = c + np.sinh(strength * tt) / math.sinh(strength)
    x = lo + (hi - lo) * (x + 1) / 2
    x[0], x[-1] = lo, hi
    return x


def stretched_grid(x: np.ndarray, y: np.ndarray, z: np.ndarray) -> Grid:
    """A stretched rectilinear grid with the given node coordinates; origin and
    spacing hold the first node and the mean cell width of each axis."""
    ax = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, z)]
    for v in ax:
        if v.size < 2 or not np.all(np.diff(v) > 0):
            raise ValueError("node coordinates must be strictly increasing")
    return Grid(ax[0].size, ax[1].size, ax[2].size, tuple(float(v[0]) for v in ax),
                tuple(float((v[-1] - v[0]) / (v.size - 1)) for v in ax), tuple(ax))


@dataclass
class Cylinder:
    """Seeds on a cylindrical mapping surface (axis along z through `centre`, radius
    r): seed (i, j) = (xc + r cos(theta0 + i dtheta), yc + r sin(theta0 + i dtheta),
    z0 + j dz), i < ntheta (fastest), j < nz."""

    centre: Tuple[float, float]
    r: float
    theta0: float
    dtheta: float
    ntheta: int
    z0: float
    dz: float
    nz: int

    def points(self) -> np.ndarray:
        th = self.theta0 + self.dtheta * np.arange(self.ntheta)
        z = self.z0 + self.dz * np.arange(self.nz)
        Z, TH = np.meshgrid(z, th, indexing="ij")
        return np.stack([self.centre[0] + self.r * np.cos(TH), self.centre[1] + self.r * np.sin(TH), Z],
                        axis=-1).reshape(-1, 3)


@dataclass
class Plane:
    """A 2-D seed grid: seed (i, j) = origin + i*du*u + j*dv*v, i < nu, j < nv.

    u and v are orthonormal; the map's squashing factor is taken on this plane (S0).
    """

    origin: Tuple[float, float, float]
    u: Tuple[float, float, float]
    v: Tuple[float, float, float]
    nu: int
    nv: int
    du: float
    dv: float

    def points(self) -> np.ndarray:
        i = np.arange(self.nu, dtype=np.float64)
        j = np.arange(self.nv, dtype=np.float64)
        jj, ii = np.meshgrid(j, i, indexing="ij")  # (nv, nu), i fastest
        o = np.asarray(self.origin)
        u = np.asarray(self.u)
        v = np.asarray(self.v)
        pts = o[None, None, :] + (ii[..., None] * self.du) * u + (jj[..., None] * self.dv) * v
        return pts.reshape(-1, 3)


@dataclass
class Voxels:
    """3-D seeds at origin + (i,j,k)*spacing, i fastest."""

    origin: Tuple[float, float, float]
    spacing: Tuple[float, float, float]
    n: Tuple[int, int, int]

    def points(self) -> np.ndarray:
        ax = [o + d * np.arange(m, dtype=np.float64) for o, d, m in
              zip(self.origin, self.spacing, self.n)]
        zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        return np.stack([xx, yy, zz], axis=-1).reshape(-1, 3)


def plane_z0(n: int, extent_x: float = 1.0, extent_y: float = 1.0) -> Plane:
    """Cell-centred n x n seeds on the bottom face z = 0: seed spacing extent/n."""
    du = extent_x / n
    dv = extent_y / n
    return Plane((0.5 * du, 0.5 * dv, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), n, n, du, dv)


# --------------------------------------------------------------------------------------
# field models
# --------------------------------------------------------------------------------------


def _node_coords(grid: Grid, k0: int, k1: int):
    x, y, z = grid.axes()
    zz, yy, xx = np.meshgrid(z[k0:k1], y, x, indexing="ij")
    return xx, yy, zz


def draw_charges(rng: np.random.Generator, n: int, xy=(0.2, 0.8), z=(-0.3, -0.1),
                 strength=(0.5, 1.5)) -> Tuple[np.ndarray, np.ndarray]:
    """Magnetic point charges below the box, with strengths that sum to zero.

    |q| ~ U(strength); the first ceil(n/2) are positive, the rest negative, and the
    negative ones are rescaled so the total charge is exactly zero (a balanced,
    flux-closing configuration).
    """
    pos = np.empty((n, 3), dtype=np.float64)
    pos[:, 0] = rng.uniform(xy[0], xy[1], n)
    pos[:, 1] = rng.uniform(xy[0], xy[1], n)
    pos[:, 2] = rng.uniform(z[0], z[1], n)
    mag = rng.uniform(strength[0], strength[1], n)
    npos = (n + 1) // 2
    q = mag.copy()
    q[npos:] *= -1.0
    if n > npos:
        q[npos:] *= q[:npos].sum() / (-q[npos:].sum())
    return pos, q


def charges_field(grid: Grid, pos: np.ndarray, q: np.ndarray, dtype=np.float64,
                  out: Optional[np.ndarray] = None, chunk: int = 16) -> np.ndarray:
    """B(r) = sum_i q_i (r - r_i) / |r - r_i|^3, the point-charge potential field of the
    paper's analytic quadrupole (Section 3.2), sampled at every node."""
    if out is None:
        out = np.zeros((3,) + grid.shape, dtype=dtype)
    for k0 in range(0, grid.nz, chunk):
        k1 = min(grid.nz, k0 + chunk)
        xx, yy, zz = _node_coords(grid, k0, k1)
        acc = np.zeros((3,) + xx.shape, dtype=np.float64)
        for (px, py, pz), qi in zip(pos, q):
            dx = xx - px
            dy = yy - py
            dz = zz - pz
            r2 = dx * dx + dy * dy + dz * dz
            f = qi / (r2 * np.sqrt(r2))
            acc[0] += f * dx
            acc[1] += f * dy
            acc[2] += f * dz
        out[:, k0:k1] += acc.astype(dtype, copy=False) if out.dtype != np.float64 else acc
    return out


def _tube_profile(rho: np.ndarray, a: float) -> np.ndarray:
    """C2 taper (1 - (rho/a)^2)^3 inside rho < a, zero outside."""
    s = np.clip(1.0 - (rho / a) ** 2, 0.0, None)
    return s * s * s


def tube_q_for_turns(R0: float, zc: float, turns: float) -> float:
    """Twist rate q (radians per unit axis length) giving `turns` turns over the part
    of the circular axis that lies above z = 0 (centre zc < 0 below the bottom face)."""
    arc = 2.0 * R0 * math.acos(min(1.0, abs(zc) / R0))
    return 2.0 * math.pi * turns / arc


def tube_field(grid: Grid, center, R0: float, a: float, B0: float, q: float,
               plane_normal: int = 1, chunk: int = 16) -> np.ndarray:
    """An arched, uniformly twisted flux tube (a torus sector).

    The tube axis is the circle of radius R0 about `center` in the plane through
    `center` normal to axis `plane_normal` (1: the x-z plane, the tube runs along x;
    0: the y-z plane, it runs along y). With R the distance from the torus symmetry
    axis and (xi, eta) = (R - R0, offset along plane_normal), rho = |(xi, eta)|:

        B = B0 (R0/R) f(rho) [ e_phi + q (-eta e_R + xi e_n) ],  f = C2 taper of radius a

    The toroidal part depends only on (R, eta) and the poloidal part derives from a
    flux function of rho, so the field is divergence-free for any taper f. The
    pitch B_theta / (rho B_phi) = q is uniform: `q` radians of twist per unit axis
    length.
    """
    out = np.zeros((3,) + grid.shape, dtype=np.float64)
    cx, cy, cz = center
    n = plane_normal
    ip = 0 if n == 1 else 1  # in-plane horizontal axis
    for k0 in range(0, grid.nz, chunk):
        k1 = min(grid.nz, k0 + chunk)
        xx, yy, zz = _node_coords(grid, k0, k1)
        h = (xx - cx) if ip == 0 else (yy - cy)  # in-plane horizontal offset
        w = zz - cz
        R = np.sqrt(h * h + w * w)
        R = np.where(R > 1e-300, R, 1e-300)
        eRh, eRw = h / R, w / R
        ephh, ephw = -eRw, eRh  # toroidal unit vector in the plane
        eta = (yy - cy) if n == 1 else (xx - cx)
        xi = R - R0
        rho = np.sqrt(xi * xi + eta * eta)
        f = _tube_profile(rho, a)
        amp = B0 * (R0 / R) * f
        bh = amp * (ephh + q * (-eta) * eRh)
        bw = amp * (ephw + q * (-eta) * eRw)
        bn = amp * (q * xi)
        comp_h = 0 if ip == 0 else 1
        out[comp_h, k0:k1] += bh
        out[2, k0:k1] += bw
        out[n, k0:k1] += bn
    return out


def linear_field(grid: Grid, M, b, dtype=np.float64) -> np.ndarray:
    """B(r) = M r + b for a 3x3 matrix M: trilinear interpolation and node-wise
    central differences reproduce such a field and its curl exactly."""
    M = np.asarray(M, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x, y, z = grid.axes()
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    out = np.empty((3,) + grid.shape, dtype=np.float64)
    for c in range(3):
        out[c] = M[c, 0] * xx + M[c, 1] * yy + M[c, 2] * zz + b[c]
    return out.astype(dtype)


QUADRUPOLE_POS = np.array([[-1.5, 0.0, -0.5], [-0.5, 0.0, -0.5], [0.5, 0.0, -0.5],
                           [1.5, 0.0, -0.5]])
QUADRUPOLE_Q = np.array([1.0, -1.0, 1.0, -1.0])


def quadrupole_field(spacing: float = 0.02, lo=(-2.5, -2.0, 0.0), hi=(2.5, 2.0, 2.5),
                     dtype=np.float64) -> Tuple[Grid, np.ndarray]:
    """The paper's analytic quadrupole (Section 3.2): four unit charges at
    x = -1.5, -0.5, 0.5, 1.5 (y = 0, z = -0.5) with alternating signs +,-,+,-,
    sampled on a uniform grid of the given spacing. The paper does not state the
    domain; the default is symmetric about x = 0 and y = 0 so that the discrete
    field keeps the mirror symmetries."""
    n = [int(round((h - l) / spacing)) + 1 for l, h in zip(lo, hi)]
    g = Grid(n[0], n[1], n[2], tuple(lo), (spacing, spacing, spacing))
    return g, charges_field(g, QUADRUPOLE_POS, QUADRUPOLE_Q, dtype=dtype)


# --------------------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    grid: Grid
    field: np.ndarray  # (3, nz, ny, nx)
    plane: Optional[Plane] = None
    voxels: Optional[Voxels] = None
    meta: dict = field(default_factory=dict)


def config_c1(seed: int = 0, nseed: int = 128) -> Workload:
    """64^3 nodes on [0,1]^3, float64: 4 seeded charges at depth 0.1-0.3 below the
    box; cell-centred 128 x 128 seeds on z = 0."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(64, 64, 64)
    pos, q = draw_charges(rng, 4)
    B = charges_field(g, pos, q, dtype=np.float64)
    return Workload("c1_quadrupolar_64", g, B, plane=plane_z0(nseed),
                    meta={"charges": (pos, q)})


def config_c1s(seed: int = 0, nseed: int = 128) -> Workload:
    """C1 on a stretched rectilinear grid: 64 x 64 x 64 nodes on [0,1]^3 with x and y
    clustered around the box centre (cells 0.67x-1.7x the mean width) and z cells
    growing by 3% per cell upward (0.35x-2.2x); float64, the same 4 seeded charges,
    cell-centred 128 x 128 seeds on z = 0."""
    rng = np.random.default_rng(seed)
    x = clustered_axis(64, 0.0, 1.0, 0.5, 1.6)
    z = geometric_axis(64, 0.0, 1.0, 1.03)
    g = stretched_grid(x, x.copy(), z)
    pos, q = draw_charges(rng, 4)
    B = charges_field(g, pos, q, dtype=np.float64)
    return Workload("c1s_quadrupolar_64_stretched", g, B, plane=plane_z0(nseed),
                    meta={"charges": (pos, q)})


def config_c2s(seed: int = 0, nseed: int = 1024) -> Workload:
    """C2 on a stretched rectilinear grid of the same node counts and box (256 x 256
    x 128 nodes on [0,1]^2 x [0, 127/255]): x and y clustered around the box centre
    (cells 0.67x-1.7x the mean width), z cells growing by 1% per cell upward
    (0.5x-1.75x); float32, the same charges and tube; 1024 x 1024 seeds on z = 0."""
    rng = np.random.default_rng(seed)
    x = clustered_axis(256, 0.0, 1.0, 0.5, 1.6)
    z = geometric_axis(128, 0.0, 127.0 / 255.0, 1.01)
    g = stretched_grid(x, x.copy(), z)
    pos, q = draw_charges(rng, 6)
    B = charges_field(g, pos, q, dtype=np.float64)
    qt = tube_q_for_turns(0.25, -0.1, 1.5)
    B += tube_field(g, (0.5, 0.5, -0.1), 0.25, 0.08, 1.0, qt, plane_normal=1)
    return Workload("c2s_charges6_tube_256x256x128_stretched", g, B.astype(np.float32),
                    plane=plane_z0(nseed), meta={"charges": (pos, q), "tube_q": qt})


def config_c2(seed: int = 0, nseed: int = 1024) -> Workload:
    """256x256x128 nodes (dx = 1/255), float32: 6 seeded charges plus one arched,
    uniformly twisted tube (R0 = 0.25, centre (0.5, 0.5, -0.1), plane y = 0.5,
    radius 0.08, B0 = 1, 1.5 turns above z = 0); 1024 x 1024 seeds on z = 0."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(256, 256, 128)
    pos, q = draw_charges(rng, 6)
    B = charges_field(g, pos, q, dtype=np.float64)
    qt = tube_q_for_turns(0.25, -0.1, 1.5)
    B += tube_field(g, (0.5, 0.5, -0.1), 0.25, 0.08, 1.0, qt, plane_normal=1)
    return Workload("c2_charges6_tube_256x256x128", g, B.astype(np.float32),
                    plane=plane_z0(nseed), meta={"charges": (pos, q), "tube_q": qt})


def c3_spec(seed: int = 0, nvox=(256, 256, 128)):
    """The draws and geometry of C3: (grid, charge positions, strengths, tubes as
    (centre, R0, a, B0, q, plane_normal), voxels, twist rate)."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(512, 512, 256)
    pos, q = draw_charges(rng, 10)
    qt = tube_q_for_turns(0.2, -0.08, 1.5)
    tubes = [((0.5, 0.35, -0.08), 0.2, 0.08, 1.0, qt, 1),
             ((0.65, 0.5, -0.08), 0.2, 0.08, 1.0, -qt, 0)]
    ux, uy, uz = g.upper
    sp = (ux / nvox[0], uy / nvox[1], uz / nvox[2])
    vox = Voxels((0.5 * sp[0], 0.5 * sp[1], 0.5 * sp[2]), sp, tuple(nvox))
    return g, pos, q, tubes, vox, qt


def config_c3(seed: int = 0, nvox=(256, 256, 128)) -> Workload:
    """512x512x256 nodes (dx = 1/511), float32: 10 seeded charges plus two arched
    tubes of opposite handedness (R0 = 0.2, centre 0.08 below z = 0, radius 0.08,
    1.5 turns; one in plane y = 0.35 along x, one in plane x = 0.65 along y);
    3-D maps on the 256x256x128 voxel centres. The charge field and each tube are
    rounded to float32 separately and summed in float32."""
    g, pos, q, tubes, vox, qt = c3_spec(seed, nvox)
    B = np.zeros((3,) + g.shape, dtype=np.float32)
    charges_field(g, pos, q, dtype=np.float32, out=B)
    for c, R0, a, B0, qq, n in tubes:
        B += tube_field(g, c, R0, a, B0, qq, plane_normal=n).astype(np.float32)
    return Workload("c3_charges10_tubes2_512x512x256", g, B, voxels=vox,
                    meta={"charges": (pos, q), "tube_q": qt})


def c4_specs(seed: int = 0, njobs: int = 16, edge=(64, 384), sides=(128, 256, 512, 1024),
             ncharge=(4, 12)) -> list:
    """The draws of the uneven batch: per cube (name, edge E, charge positions,
    strengths, seed-grid side)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(njobs):
        E = int(rng.integers(edge[0], edge[1] + 1))
        nc = int(rng.integers(ncharge[0], ncharge[1] + 1))
        side = int(rng.choice(np.asarray(sides)))
        pos, q = draw_charges(rng, nc)
        out.append((f"c4_job{j}_E{E}_S{side}", E, pos, q, side))
    return out


def config_c4(seed: int = 0, njobs: int = 16, edge=(64, 384), sides=(128, 256, 512, 1024),
              ncharge=(4, 12)) -> List[Workload]:
    """Uneven batch: per cube an edge E ~ U{64..384} (cubic, dx = 1/(E-1)), float32,
    U{4..12} seeded charges, and a seed-grid side drawn from {128, 256, 512, 1024}
    on z = 0."""
    jobs = []
    for name, E, pos, q, side in c4_specs(seed, njobs, edge, sides, ncharge):
        g = cubic_grid(E, E, E)
        B = np.zeros((3,) + g.shape, dtype=np.float32)
        charges_field(g, pos, q, dtype=np.float32, out=B)
        jobs.append(Workload(name, g, B, plane=plane_z0(side), meta={"charges": (pos, q)}))
    return jobs


def config_c5(seed: int = 0, nseed: int = 256) -> Tuple[Workload, dict]:
    """128x128x96 nodes (dx = 1/127), float32, 8 seeded charges (the learnable start)
    and a second seeded 8-charge field (the target); 256 x 256 seeds on z = 0."""
    rng = np.random.default_rng(seed)
    g = cubic_grid(128, 128, 96)
    pos, q = draw_charges(rng, 8)
    tpos, tq = draw_charges(rng, 8)
    B = charges_field(g, pos, q, dtype=np.float32)
    Bt = charges_field(g, tpos, tq, dtype=np.float32)
    w = Workload("c5_adjoint_128x128x96", g, B, plane=plane_z0(nseed),
                 meta={"charges": (pos, q)})
    return w, {"field": Bt, "charges": (tpos, tq)}
