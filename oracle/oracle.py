"""ctypes wrapper of the FP64 C oracle (``fq_oracle.c``). Test infrastructure only."""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fq_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ORC_OK = 0
ORC_OUTSIDE = 1
ORC_NULLB = 2
ORC_MAXSTEPS = 4
ORC_NONFINITE = 8
ORC_ONESIDED = 16
ORC_MIXEDFACE = 32
ORC_EDGE = 64
ORC_ROTATED = 128
FATAL = ORC_OUTSIDE | ORC_NULLB | ORC_MAXSTEPS | ORC_NONFINITE


class _Field(C.Structure):
    _fields_ = [
        ("n", C.c_int64 * 3),
        ("origin", C.c_double * 3),
        ("spacing", C.c_double * 3),
        ("b", C.c_void_p * 3),
        ("j", C.c_void_p * 3),
        ("coord", C.c_void_p * 3),
    ]


class _Cyl(C.Structure):
    _fields_ = [("xc", C.c_double), ("yc", C.c_double), ("r", C.c_double)]


ORC_FACE_CYL = 6


class _Opts(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("h0", C.c_double),
        ("hmax", C.c_double),
        ("max_steps", C.c_int64),
        ("edge_eps", C.c_double),
        ("want_tw", C.c_int),
        ("nthreads", C.c_int),
    ]


class _Lines(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("end_b", "end_f", "face_b", "face_f", "bn_b", "bn_f", "bn0", "tw", "len",
                 "status", "nsteps")]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, OpenMP; no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        lib.orc_curl.argtypes = [C.POINTER(_Field), C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_interp.argtypes = [C.POINTER(_Field), C.c_void_p * 3, C.c_int64 * 3,
                                   C.c_double * 3, C.c_double * 3]
        lib.orc_trace.argtypes = [C.POINTER(_Field), C.c_void_p, C.c_int64, C.c_void_p,
                                  C.POINTER(_Opts), C.POINTER(_Lines)]
        lib.orc_q2d.argtypes = [C.POINTER(_Field), C.c_double * 3, C.c_double * 3,
                                C.c_double * 3, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                C.POINTER(_Opts), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.POINTER(_Lines)]
        lib.orc_q3d.argtypes = [C.POINTER(_Field), C.c_double * 3, C.c_double * 3,
                                C.c_int64 * 3, C.POINTER(_Opts), C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.POINTER(_Lines)]
        lib.orc_method2.argtypes = [C.POINTER(_Field), C.c_void_p, C.c_int64, C.c_int,
                                    C.POINTER(_Opts), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.POINTER(_Lines)]
        lib.orc_q2d_perp.argtypes = [C.POINTER(_Field), C.c_double * 3, C.c_double * 3,
                                     C.c_double * 3, C.c_int64, C.c_int64, C.c_double,
                                     C.c_double, C.POINTER(_Opts), C.c_void_p, C.c_void_p,
                                     C.c_void_p]
        lib.orc_qcyl.argtypes = [C.POINTER(_Field), C.POINTER(_Cyl), C.c_double, C.c_double,
                                 C.c_int64, C.c_double, C.c_double, C.c_int64, C.POINTER(_Opts),
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_default_opts.argtypes = [C.POINTER(_Opts)]
        lib.orc_threads.restype = C.c_int
        lib.orc_q2d_points.argtypes = [C.POINTER(_Field), C.c_double * 3, C.c_double * 3,
                                       C.c_double * 3, C.c_int64, C.c_int64, C.c_double,
                                       C.c_double, C.c_void_p, C.c_int64, C.POINTER(_Opts),
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.POINTER(_Lines)]
        lib.orc_q3d_points.argtypes = [C.POINTER(_Field), C.c_double * 3, C.c_double * 3,
                                       C.c_int64 * 3, C.c_void_p, C.c_int64, C.POINTER(_Opts),
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.POINTER(_Lines)]
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_threads())


def default_opts(**kw) -> dict:
    o = _Opts()
    _load().orc_default_opts(C.byref(o))
    d = {k: getattr(o, k) for k, _ in _Opts._fields_}
    d.update(kw)
    return d


def _opts(kw: Optional[dict]) -> _Opts:
    d = default_opts(**(kw or {}))
    o = _Opts()
    for k, _ in _Opts._fields_:
        setattr(o, k, d[k])
    return o


class _FieldHolder:
    """Keeps the float64 planes (and curl planes) alive while C uses them."""

    def __init__(self, B: np.ndarray, grid, want_curl: bool = True):
        lib = _load()
        self.b = [np.ascontiguousarray(B[c], dtype=np.float64) for c in range(3)]
        nz, ny, nx = self.b[0].shape
        f = _Field()
        f.n[:] = (nx, ny, nz)
        f.origin[:] = tuple(float(x) for x in grid.origin)
        f.spacing[:] = tuple(float(x) for x in grid.spacing)
        # stretched axes: node coordinates (kept alive here)
        self.coord = [grid.coord(a) if hasattr(grid, "coord") else None for a in range(3)]
        for a in range(3):
            f.coord[a] = self.coord[a].ctypes.data if self.coord[a] is not None else None
        for c in range(3):
            f.b[c] = self.b[c].ctypes.data
        self.j = [np.zeros_like(self.b[0]) for _ in range(3)]
        for c in range(3):
            f.j[c] = self.j[c].ctypes.data
        self.f = f
        if want_curl:
            rc = lib.orc_curl(C.byref(f), *(a.ctypes.data for a in self.j))
            if rc != 0:
                raise ValueError("oracle curl: grid needs at least 2 nodes per axis")


def curl(B: np.ndarray, grid) -> np.ndarray:
    h = _FieldHolder(B, grid)
    return np.stack(h.j)


def interp(B: np.ndarray, grid, cell, r) -> np.ndarray:
    """Trilinear interpolant of B in `cell` at point r (r may lie outside the cell:
    the cell's polynomial is extended)."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=False)
    planes = (C.c_void_p * 3)(*[h.f.b[c] for c in range(3)])
    out = (C.c_double * 3)()
    lib.orc_interp(C.byref(h.f), planes, (C.c_int64 * 3)(*cell), (C.c_double * 3)(*r), out)
    return np.array(out[:])


def _lines_struct(n: int):
    arrs = {
        "end_b": np.full((n, 3), np.nan), "end_f": np.full((n, 3), np.nan),
        "face_b": np.full(n, -1, np.int8), "face_f": np.full(n, -1, np.int8),
        "bn_b": np.full(n, np.nan), "bn_f": np.full(n, np.nan), "bn0": np.full(n, np.nan),
        "tw": np.full(n, np.nan), "len": np.full(n, np.nan),
        "status": np.zeros(n, np.uint16), "nsteps": np.zeros(n, np.int64),
    }
    s = _Lines()
    for k, a in arrs.items():
        setattr(s, k, a.ctypes.data)
    return s, arrs


def trace(B: np.ndarray, grid, seeds: np.ndarray, normal=(0.0, 0.0, 1.0),
          opts: Optional[dict] = None) -> dict:
    """Trace every seed both ways; returns per-line arrays."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    n = seeds.shape[0]
    s, arrs = _lines_struct(n)
    nrm = np.ascontiguousarray(normal, dtype=np.float64)
    o = _opts(opts)
    lib.orc_trace(C.byref(h.f), seeds.ctypes.data, n, nrm.ctypes.data, C.byref(o), C.byref(s))
    return arrs


def q2d(B: np.ndarray, grid, plane, opts: Optional[dict] = None, want_lines: bool = True) -> dict:
    """Q, Tw, length and status on a 2-D seed grid (shape (nv, nu), u fastest)."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    n = plane.nu * plane.nv
    out = {"q": np.full(n, np.nan), "tw": np.full(n, np.nan), "len": np.full(n, np.nan),
           "status": np.zeros(n, np.uint16)}
    s, arrs = _lines_struct(n) if want_lines else (None, {})
    o = _opts(opts)
    rc = lib.orc_q2d(C.byref(h.f), (C.c_double * 3)(*plane.origin), (C.c_double * 3)(*plane.u),
                     (C.c_double * 3)(*plane.v), plane.nu, plane.nv, plane.du, plane.dv,
                     C.byref(o), out["q"].ctypes.data, out["tw"].ctypes.data,
                     out["len"].ctypes.data, out["status"].ctypes.data,
                     C.byref(s) if s is not None else None)
    if rc != 0:
        raise RuntimeError(f"orc_q2d failed: {rc}")
    out["lines"] = arrs
    shp = (plane.nv, plane.nu)
    for k in ("q", "tw", "len", "status"):
        out[k] = out[k].reshape(shp)
    return out


def q3d(B: np.ndarray, grid, vox, opts: Optional[dict] = None, want_lines: bool = True) -> dict:
    """3-D Q, Tw, length and status on voxel centres (shape (nz, ny, nx))."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    n = int(np.prod(vox.n))
    out = {"q": np.full(n, np.nan), "tw": np.full(n, np.nan), "len": np.full(n, np.nan),
           "status": np.zeros(n, np.uint16)}
    s, arrs = _lines_struct(n) if want_lines else (None, {})
    o = _opts(opts)
    rc = lib.orc_q3d(C.byref(h.f), (C.c_double * 3)(*vox.origin),
                     (C.c_double * 3)(*vox.spacing), (C.c_int64 * 3)(*vox.n), C.byref(o),
                     out["q"].ctypes.data, out["tw"].ctypes.data, out["len"].ctypes.data,
                     out["status"].ctypes.data, C.byref(s) if s is not None else None)
    if rc != 0:
        raise RuntimeError(f"orc_q3d failed: {rc}")
    out["lines"] = arrs
    shp = (vox.n[2], vox.n[1], vox.n[0])
    for k in ("q", "tw", "len", "status"):
        out[k] = out[k].reshape(shp)
    return out


def _points_out(n):
    return {"q": np.full(n, np.nan), "tw": np.full(n, np.nan), "len": np.full(n, np.nan),
            "status": np.zeros(n, np.uint16)}


def q2d_points(B: np.ndarray, grid, plane, pts, opts: Optional[dict] = None) -> dict:
    """Q, Tw, length, status and the point's own line at listed map points
    (flat indices, i fastest), each traced with its stencil neighbours."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    n = pts.size
    out = _points_out(n)
    s, arrs = _lines_struct(n)
    o = _opts(opts)
    rc = lib.orc_q2d_points(C.byref(h.f), (C.c_double * 3)(*plane.origin),
                            (C.c_double * 3)(*plane.u), (C.c_double * 3)(*plane.v), plane.nu,
                            plane.nv, plane.du, plane.dv, pts.ctypes.data, n, C.byref(o),
                            out["q"].ctypes.data, out["tw"].ctypes.data, out["len"].ctypes.data,
                            out["status"].ctypes.data, C.byref(s))
    if rc != 0:
        raise ValueError("orc_q2d_points: point index out of range")
    out["lines"] = arrs
    return out


def q3d_points(B: np.ndarray, grid, vox, pts, opts: Optional[dict] = None) -> dict:
    """3-D map values at listed voxels (flat indices, i fastest)."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    n = pts.size
    out = _points_out(n)
    s, arrs = _lines_struct(n)
    o = _opts(opts)
    rc = lib.orc_q3d_points(C.byref(h.f), (C.c_double * 3)(*vox.origin),
                            (C.c_double * 3)(*vox.spacing), (C.c_int64 * 3)(*vox.n),
                            pts.ctypes.data, n, C.byref(o), out["q"].ctypes.data,
                            out["tw"].ctypes.data, out["len"].ctypes.data,
                            out["status"].ctypes.data, C.byref(s))
    if rc != 0:
        raise ValueError("orc_q3d_points: point index out of range")
    out["lines"] = arrs
    return out


def qcyl(B: np.ndarray, grid, cyl, opts: Optional[dict] = None) -> dict:
    """Q, Tw, length, status (shape (nz, ntheta), theta fastest) and lines on a
    cylindrical mapping surface; `cyl` has centre (xc, yc), r, theta0, dtheta, ntheta,
    z0, dz, nz (synth.Cylinder)."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    n = cyl.ntheta * cyl.nz
    out = {"q": np.full(n, np.nan), "tw": np.full(n, np.nan), "len": np.full(n, np.nan),
           "status": np.zeros(n, np.uint16)}
    s, arrs = _lines_struct(n)
    c = _Cyl(float(cyl.centre[0]), float(cyl.centre[1]), float(cyl.r))
    rc = lib.orc_qcyl(C.byref(h.f), C.byref(c), float(cyl.theta0), float(cyl.dtheta), int(cyl.ntheta),
                      float(cyl.z0), float(cyl.dz), int(cyl.nz), C.byref(_opts(opts)),
                      out["q"].ctypes.data, out["tw"].ctypes.data, out["len"].ctypes.data,
                      out["status"].ctypes.data, C.byref(s))
    if rc != 0:
        raise RuntimeError(f"orc_qcyl failed: {rc}")
    for k in ("q", "tw", "len", "status"):
        out[k] = out[k].reshape(cyl.nz, cyl.ntheta)
    out["lines"] = arrs
    return out


def q2d_perp(B: np.ndarray, grid, plane, opts: Optional[dict] = None) -> dict:
    """Method I Q_perp (S1, S2 perpendicular to B at the ends) and the length edge map
    |grad_S0 length| on a 2-D seed grid (shape (nv, nu), u fastest), with statuses."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=False)
    n = plane.nu * plane.nv
    out = {"qperp": np.full(n, np.nan), "fledge": np.full(n, np.nan),
           "status": np.zeros(n, np.uint16)}
    o = _opts(dict(opts or {}, want_tw=0))
    rc = lib.orc_q2d_perp(C.byref(h.f), (C.c_double * 3)(*plane.origin), (C.c_double * 3)(*plane.u),
                          (C.c_double * 3)(*plane.v), plane.nu, plane.nv, plane.du, plane.dv,
                          C.byref(o), out["qperp"].ctypes.data, out["fledge"].ctypes.data,
                          out["status"].ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_q2d_perp failed: {rc}")
    for k in out:
        out[k] = out[k].reshape(plane.nv, plane.nu)
    return out


def method2(B: np.ndarray, grid, seeds: np.ndarray, way: int = 2,
            opts: Optional[dict] = None) -> dict:
    """Method II at every seed (n x 3): Q (S1, S2 = the faces the line ends on),
    Q_perp (S1, S2 perpendicular to B), Tw, length, status and the ends. way 1 takes
    grad(B/B) from node values, way 2 from offset differences."""
    lib = _load()
    h = _FieldHolder(B, grid, want_curl=(opts or {}).get("want_tw", 1) != 0)
    seeds = np.ascontiguousarray(seeds, dtype=np.float64).reshape(-1, 3)
    n = seeds.shape[0]
    out = {"q": np.full(n, np.nan), "qperp": np.full(n, np.nan), "tw": np.full(n, np.nan),
           "len": np.full(n, np.nan), "status": np.zeros(n, np.uint16)}
    s, arrs = _lines_struct(n)
    o = _opts(opts)
    rc = lib.orc_method2(C.byref(h.f), seeds.ctypes.data, n, int(way), C.byref(o),
                         out["q"].ctypes.data, out["qperp"].ctypes.data, out["tw"].ctypes.data,
                         out["len"].ctypes.data, out["status"].ctypes.data, C.byref(s))
    if rc != 0:
        raise ValueError(f"orc_method2 failed: {rc}")
    out["lines"] = arrs
    return out
