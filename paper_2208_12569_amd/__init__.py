"""MI355X field-line tracer for the squashing factor Q and the twist number Tw.

Python binding of libfastqsl.so (include/fastqsl.h). This layer only marshals
arguments: PyTorch provides device memory and the stream, and every step of the
computation runs in the library's HIP kernels. There is no CPU fallback; calls fail
if the library is missing or no GPU is present.

Fields are torch tensors of shape (3, nz, ny, nx) (Bx, By, Bz planes, x fastest),
float32 or float64, on the current CUDA/HIP device. `grid` is any object with
`origin` and `spacing` 3-sequences (node (i,j,k) at origin + (i,j,k)*spacing).
"""

from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (  # noqa: F401
    FQ_PREC_F32X,
    FQ_PREC_F64,
    FQ_METHOD_I,
    FQ_METHOD_II,
    FQ_FACE_CYL,
    FQ_SCHEME_RK4,
    FQ_SCHEME_RK4_38,
    FQ_SCHEME_RKF45,
    ST_EDGE,
    ST_FATAL,
    ST_MAXSTEPS,
    ST_MIXEDFACE,
    ST_NONFINITE,
    ST_NOTAPE,
    ST_NULLB,
    ST_ONESIDED,
    ST_OUTSIDE,
    ST_ROTATED,
)


@dataclass
class Params:
    """Tracing parameters (zero = library default; see fq_params in fastqsl.h)."""

    tol_perp: float = 0.0
    step_perp: float = 0.0
    step_min: float = 0.0
    tol_floor: float = 0.0
    edge_eps: float = 0.0
    max_steps: int = 0
    precision: int = FQ_PREC_F32X
    want_tw: bool = True
    block: int = 0
    waves_per_cu: int = 0
    graze: float = 0.0
    qfix: float = 0.0
    tape_steps: int = 0  # adjoint calls: checkpoint pool room in accepted steps per half line
    scheme: int = FQ_SCHEME_RKF45
    method: int = FQ_METHOD_I  # maps: FQ_METHOD_II adds Q_perp ("qperp")
    in_flight: bool = False  # F32X maps: other maps run on other streams at the same time
    stats: object = None  # optional CUDA int64 tensor of 5 counters (added to)
    events: object = None  # optional ctypes array of 4 hipEvent_t handles

    def c(self) -> _lib.fq_params:
        p = _lib.fq_params()
        p.tol_perp = self.tol_perp
        p.step_perp = self.step_perp
        p.step_min = self.step_min
        p.tol_floor = self.tol_floor
        p.edge_eps = self.edge_eps
        p.max_steps = int(self.max_steps)
        p.precision = int(self.precision)
        p.want_tw = 1 if self.want_tw else 0
        p.block = int(self.block)
        p.waves_per_cu = int(self.waves_per_cu)
        p.graze = float(self.graze)
        p.qfix = float(self.qfix)
        p.tape_steps = int(self.tape_steps)
        p.scheme = int(self.scheme)
        p.method = int(self.method)
        p.in_flight = 1 if self.in_flight else 0
        p.stats = self.stats.data_ptr() if self.stats is not None else None
        p.events = C.cast(self.events, C.c_void_p) if self.events is not None else None
        return p


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("paper_2208_12569_amd needs a GPU (no CPU fallback)")
    return torch


def _stream(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _field(B, grid) -> _lib.fq_field:
    torch = _torch()
    if B.dim() != 4 or B.shape[0] != 3 or not B.is_cuda:
        raise ValueError("B must be a CUDA tensor of shape (3, nz, ny, nx)")
    if B.dtype not in (torch.float32, torch.float64):
        raise ValueError("B must be float32 or float64")
    if not B.is_contiguous():
        raise ValueError("B must be contiguous")
    f = _lib.fq_field()
    nz, ny, nx = B.shape[1:]
    f.n[:] = (nx, ny, nz)
    f.origin[:] = tuple(float(v) for v in grid.origin)
    f.spacing[:] = tuple(float(v) for v in grid.spacing)
    f.dtype = _lib.FQ_DT_F32 if B.dtype == torch.float32 else _lib.FQ_DT_F64
    for c in range(3):
        f.b[c] = B[c].data_ptr()
    for a, t in enumerate(_coords(grid, B.device)):
        f.coord[a] = t.data_ptr() if t is not None else None
    return f


def _coords(grid, device):
    """Device FP64 node coordinates of a grid's stretched axes (None per uniform
    axis). A grid may carry them as CUDA tensors already; numpy coordinates are
    copied once per device and kept on the grid object, so their device memory
    lives as long as the grid (the library reads them asynchronously, also from
    captured graphs)."""
    torch = _torch()
    coords = getattr(grid, "coords", None)
    if coords is None:
        return (None, None, None)
    cache = grid.__dict__.setdefault("_fq_device_coords", {})
    out = []
    for a in range(3):
        c = coords[a]
        if c is None:
            out.append(None)
            continue
        if isinstance(c, torch.Tensor) and c.is_cuda:
            if c.dtype != torch.float64 or not c.is_contiguous() or c.device != device:
                raise ValueError("device node coordinates must be contiguous float64 on B's device")
            out.append(c)
            continue
        key = (str(device), a)
        if key not in cache:
            cache[key] = torch.as_tensor(np.ascontiguousarray(c, dtype=np.float64)).to(device)
        out.append(cache[key])
    return tuple(out)


def _plane(pl) -> _lib.fq_plane:
    p = _lib.fq_plane()
    p.origin[:] = tuple(float(v) for v in pl.origin)
    p.u[:] = tuple(float(v) for v in pl.u)
    p.v[:] = tuple(float(v) for v in pl.v)
    p.nu, p.nv = int(pl.nu), int(pl.nv)
    p.du, p.dv = float(pl.du), float(pl.dv)
    return p


def _voxels(vx) -> _lib.fq_voxels:
    v = _lib.fq_voxels()
    v.origin[:] = tuple(float(x) for x in vx.origin)
    v.spacing[:] = tuple(float(x) for x in vx.spacing)
    v.n[:] = tuple(int(x) for x in vx.n)
    return v


_LINE_KEYS = ("end_b", "end_f", "face_b", "face_f", "bn_b", "bn_f", "bn0", "tw", "length", "status")


def _alloc_lines(n: int, device, keys=_LINE_KEYS):
    torch = _torch()
    out = {}
    for k in keys:
        if k in ("end_b", "end_f"):
            out[k] = torch.empty((n, 3), dtype=torch.float64, device=device)
        elif k in ("face_b", "face_f"):
            out[k] = torch.empty(n, dtype=torch.int8, device=device)
        elif k == "status":
            out[k] = torch.empty(n, dtype=torch.int16, device=device)
        else:
            out[k] = torch.empty(n, dtype=torch.float64, device=device)
    return out


def _lines_struct(d: dict) -> _lib.fq_lines:
    s = _lib.fq_lines()
    for k in _LINE_KEYS:
        if k in d:
            setattr(s, k, d[k].data_ptr())
    return s


def _workspace(nbytes: int, device, ws=None):
    torch = _torch()
    if ws is not None and ws.numel() >= nbytes:
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def version() -> str:
    return _lib.load().fastqsl_version().decode()


def trace(B, grid, seeds, normal=(0.0, 0.0, 1.0), params: Optional[Params] = None,
          stream=None, ws=None) -> dict:
    """Trace every seed (a CUDA float64 tensor of shape (n, 3)) both ways to the box."""
    torch = _torch()
    lib = _lib.load()
    params = params or Params()
    f = _field(B, grid)
    p = params.c()
    seeds = seeds.to(device=B.device, dtype=torch.float64).contiguous()
    n = seeds.shape[0]
    out = _alloc_lines(n, B.device)
    need = lib.fastqsl_trace_workspace_size(C.byref(f), n, C.byref(p))
    if need == 0:
        raise ValueError("invalid field or parameters")
    w = _workspace(need, B.device, ws)
    nrm = (C.c_double * 3)(*normal)
    ls = _lines_struct(out)
    _lib.check(lib.fastqsl_trace(C.byref(f), seeds.data_ptr(), n, nrm, C.byref(p), C.byref(ls),
                                 w.data_ptr(), w.numel(), _stream(stream)), "fastqsl_trace")
    out["_ws"] = w
    return out


def _alloc_map(npts: int, shape, device, want_lines: bool, qperp: bool = False,
               fledge: bool = False):
    torch = _torch()
    m = {"q": torch.empty(shape, dtype=torch.float64, device=device),
         "tw": torch.empty(shape, dtype=torch.float64, device=device),
         "length": torch.empty(shape, dtype=torch.float64, device=device),
         "status": torch.empty(shape, dtype=torch.int16, device=device)}
    s = _lib.fq_map()
    s.q = m["q"].data_ptr()
    s.tw = m["tw"].data_ptr()
    s.length = m["length"].data_ptr()
    s.status = m["status"].data_ptr()
    if qperp:
        m["qperp"] = torch.empty(shape, dtype=torch.float64, device=device)
        s.qperp = m["qperp"].data_ptr()
    if fledge:
        m["fledge"] = torch.empty(shape, dtype=torch.float64, device=device)
        s.fledge = m["fledge"].data_ptr()
    if want_lines:
        m["lines"] = _alloc_lines(npts, device)
        s.lines = _lines_struct(m["lines"])
    return m, s


def _batch_args(jobs, params: Params, outs: list):
    n = len(jobs)
    fields = (_lib.fq_field * n)()
    planes = (_lib.fq_plane * n)()
    maps = (_lib.fq_map * n)()
    for j, (B, grid, pl) in enumerate(jobs):
        fields[j] = _field(B, grid)
        planes[j] = _plane(pl)
        m = outs[j]
        s = _lib.fq_map()
        s.q = m["q"].data_ptr()
        s.tw = m["tw"].data_ptr()
        s.length = m["length"].data_ptr()
        s.status = m["status"].data_ptr()
        if "lines" in m:
            s.lines = _lines_struct(m["lines"])
        if "qperp" in m:
            s.qperp = m["qperp"].data_ptr()
        if "fledge" in m:
            s.fledge = m["fledge"].data_ptr()
        maps[j] = s
    return fields, planes, maps, params.c()


def q2d_workspace_size(jobs: Sequence, params: Optional[Params] = None) -> int:
    """Workspace bytes fastqsl_q2d needs for these (B, grid, plane) jobs."""
    lib = _lib.load()
    params = params or Params()
    n = len(jobs)
    fields = (_lib.fq_field * n)()
    planes = (_lib.fq_plane * n)()
    for j, (B, grid, pl) in enumerate(jobs):
        fields[j] = _field(B, grid)
        planes[j] = _plane(pl)
    p = params.c()
    need = lib.fastqsl_q2d_workspace_size(fields, planes, n, C.byref(p))
    if need == 0:
        raise ValueError("invalid field, plane or parameters (or an unsupported combination)")
    return int(need)


def alloc_q2d_outputs(jobs: Sequence, want_lines: bool = False, qperp: bool = False,
                      fledge: bool = False) -> list:
    """Output maps for q2d_batch_into (one dict of CUDA tensors per job; with qperp,
    a Q_perp map too; with fledge, the length edge map)."""
    outs = []
    for B, grid, pl in jobs:
        m, _ = _alloc_map(pl.nu * pl.nv, (pl.nv, pl.nu), B.device, want_lines, qperp, fledge)
        outs.append(m)
    return outs


def q2d_batch_into(jobs: Sequence, outs: list, ws, params: Optional[Params] = None,
                   stream=None) -> None:
    """fastqsl_q2d on preallocated outputs and workspace: no allocation, no
    synchronisation, so the call can be captured into a HIP graph."""
    lib = _lib.load()
    params = params or Params()
    fields, planes, maps, p = _batch_args(jobs, params, outs)
    _lib.check(lib.fastqsl_q2d(fields, planes, len(jobs), C.byref(p), maps, ws.data_ptr(),
                               ws.numel(), _stream(stream)), "fastqsl_q2d")


def q2d_batch(jobs: Sequence, params: Optional[Params] = None, want_lines: bool = False,
              stream=None, ws=None, perp: bool = False) -> list:
    """Q/Tw/length maps for several (B, grid, plane) triples in ONE persistent launch.
    perp: also Q_perp ("qperp"; Method II always gives it) and the length edge map
    ("fledge")."""
    params = params or Params()
    need = q2d_workspace_size(jobs, params)
    w = _workspace(need, jobs[0][0].device, ws)
    outs = alloc_q2d_outputs(jobs, want_lines, perp or params.method == FQ_METHOD_II, perp)
    q2d_batch_into(jobs, outs, w, params, stream)
    for m in outs:
        m["_ws"] = w
    return outs


def q2d(B, grid, plane, params: Optional[Params] = None, want_lines: bool = False,
        stream=None, ws=None, perp: bool = False) -> dict:
    """Q, Tw and length maps on a 2-D seed grid (shape (nv, nu)); perp: Q_perp and the
    length edge map too."""
    return q2d_batch([(B, grid, plane)], params, want_lines, stream, ws, perp)[0]


_SIDE_STREAMS: dict = {}


def q2d_many(jobs: Sequence, params: Optional[Params] = None, want_lines: bool = False,
             streams: int = 4) -> list:
    """q2d maps of many (B, grid, plane) jobs, `streams` of them in flight at once on as
    many streams of default priority (the caller's current stream and streams - 1
    more; the GPU runs four hardware queues by default, and streams beyond them share
    one), each with its own workspace, in_flight set: one map's FP64 pass overlaps the
    next maps' FP32 passes (more maps per second than one call after another; the same
    maps bit for bit). The caller's current stream waits for all of them before this
    returns, so the results are ready in its order."""
    import dataclasses

    torch = _torch()
    params = dataclasses.replace(params or Params(), in_flight=True)
    n = max(1, int(streams))
    main = torch.cuda.current_stream()
    # side streams are made once per device and kept: HIP assigns hardware queues to
    # streams in the order they are created, so streams made anew for every call would
    # come to share a queue with the caller's
    side = _SIDE_STREAMS.setdefault(main.device, [])
    while len(side) < n - 1:
        side.append(torch.cuda.Stream(device=main.device))
    pool = [main] + side[:n - 1]
    start = torch.cuda.Event()
    start.record(main)
    wss: dict = {}
    out = []
    for k, (B, grid, plane) in enumerate(jobs):
        s = pool[k % n]
        s.wait_event(start)  # inputs written on the caller's stream are ready
        with torch.cuda.stream(s):
            r = q2d(B, grid, plane, params, want_lines, stream=s, ws=wss.get(k % n))
        need = int(r["_ws"].numel())
        if k % n not in wss or wss[k % n].numel() < need:
            wss[k % n] = r["_ws"]
        out.append(r)
    for s in pool[1:]:
        e = torch.cuda.Event()
        e.record(s)
        main.wait_event(e)
    # tensors made on the side streams are used on the caller's stream from now on
    for r in out:
        for v in list(r.values()) + list(r.get("lines", {}).values()):
            if hasattr(v, "record_stream"):
                v.record_stream(main)
    return out


def q2d_static(jobs: Sequence, params: Optional[Params] = None, outs: Optional[list] = None,
               want_lines: bool = False, stream=None) -> list:
    """fastqsl_q2d_static: the maps of q2d_batch with the library's own device
    scratch (no workspace is allocated; outputs are, unless `outs` from
    alloc_q2d_outputs is given). Raises if the jobs need more scratch than
    fastqsl_static_scratch_bytes()."""
    lib = _lib.load()
    params = params or Params()
    jobs = list(jobs)
    if outs is None:
        outs = alloc_q2d_outputs(jobs, want_lines)
    f, pl, m, p = _batch_args(jobs, params, outs)
    _lib.check(lib.fastqsl_q2d_static(f, pl, len(jobs), C.byref(p), m, _stream(stream)),
               "fastqsl_q2d_static")
    return outs


def static_scratch_bytes() -> int:
    return int(_lib.load().fastqsl_static_scratch_bytes())


def q3d(B, grid, voxels, params: Optional[Params] = None, want_lines: bool = False,
        stream=None, ws=None) -> dict:
    """Q, Tw and length at voxel centres (shape (nz, ny, nx) of the voxel grid)."""
    lib = _lib.load()
    params = params or Params()
    f = _field(B, grid)
    v = _voxels(voxels)
    nx, ny, nz = (int(x) for x in voxels.n)
    m, s = _alloc_map(nx * ny * nz, (nz, ny, nx), B.device, want_lines,
                      params.method == FQ_METHOD_II)
    p = params.c()
    need = lib.fastqsl_q3d_workspace_size(C.byref(f), C.byref(v), C.byref(p))
    if need == 0:
        raise ValueError("invalid field, voxels or parameters")
    w = _workspace(need, B.device, ws)
    _lib.check(lib.fastqsl_q3d(C.byref(f), C.byref(v), C.byref(p), C.byref(s), w.data_ptr(),
                               w.numel(), _stream(stream)), "fastqsl_q3d")
    m["_ws"] = w
    return m


def qcyl(B, grid, cyl, params: Optional[Params] = None, want_lines: bool = False,
         stream=None, ws=None) -> dict:
    """Q, Tw and length on a cylindrical mapping surface (shape (nz, ntheta), theta
    fastest); `cyl` has centre, r, theta0, dtheta, ntheta, z0, dz, nz."""
    lib = _lib.load()
    params = params or Params()
    f = _field(B, grid)
    c = _lib.fq_cylinder()
    c.centre[:] = (float(cyl.centre[0]), float(cyl.centre[1]))
    c.radius = float(cyl.r)
    c.theta0, c.dtheta, c.ntheta = float(cyl.theta0), float(cyl.dtheta), int(cyl.ntheta)
    c.z0, c.dz, c.nz = float(cyl.z0), float(cyl.dz), int(cyl.nz)
    m, s = _alloc_map(c.ntheta * c.nz, (c.nz, c.ntheta), B.device, want_lines)
    p = params.c()
    need = lib.fastqsl_qcyl_workspace_size(C.byref(f), C.byref(c), C.byref(p))
    if need == 0:
        raise ValueError("invalid field, cylinder or parameters (or an unsupported combination)")
    w = _workspace(need, B.device, ws)
    _lib.check(lib.fastqsl_qcyl(C.byref(f), C.byref(c), C.byref(p), C.byref(s), w.data_ptr(),
                                w.numel(), _stream(stream)), "fastqsl_qcyl")
    m["_ws"] = w
    return m


def _is_voxels(target) -> bool:
    return hasattr(target, "n") and not hasattr(target, "nu")


def _bwd_prepare(B, grid, target, params: Optional[Params], segment: int):
    """Checks and workspace size of an adjoint call on a seed plane or a voxel map."""
    lib = _lib.load()
    params = params or Params(precision=FQ_PREC_F64)
    f = _field(B, grid)
    p = params.c()
    if _is_voxels(target):
        t = _voxels(target)
        need = lib.fastqsl_q3d_backward_workspace_size(C.byref(f), C.byref(t), C.byref(p),
                                                       int(segment))
    else:
        t = _plane(target)
        need = lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(t), C.byref(p), int(segment))
    if need == 0:
        raise ValueError("invalid or unsupported backward call (Method I; RKF45 where S0 may "
                         "rotate; 1 <= segment <= 4096)")
    return lib, f, t, p, need


def _npoints(target) -> int:
    if _is_voxels(target):
        return math.prod(int(x) for x in target.n)
    return int(target.nu) * int(target.nv)


def _bwd_reverse(name, B, grid, target, params, segment, dq, dtw, dend_b, dend_f, gb, stream, ws):
    torch = _torch()
    lib, f, t, p, need = _bwd_prepare(B, grid, target, params, segment)
    if gb is None:
        gb = torch.zeros(B.shape, dtype=torch.float64, device=B.device)
    if gb.dtype != torch.float64 or gb.shape != B.shape or not gb.is_contiguous():
        raise ValueError("gb must be a contiguous float64 tensor shaped like B")
    npts = _npoints(target)

    def arg(x, shape):
        if x is None:
            return None, None
        x = x.to(device=B.device, dtype=torch.float64).contiguous()
        if x.numel() != math.prod(shape):
            raise ValueError(f"gradient of shape {tuple(x.shape)} does not fit {shape}")
        return x, x.data_ptr()

    dq_t, dq_p = arg(dq, (npts,))
    dtw_t, dtw_p = arg(dtw, (npts,))
    db_t, db_p = arg(dend_b, (npts, 3))
    df_t, df_p = arg(dend_f, (npts, 3))
    if name.endswith("_recorded") and (ws is None or ws.numel() < need):
        raise ValueError("the record does not belong to these inputs (workspace too small)")
    w = _workspace(need, B.device, ws)
    g3 = (C.c_void_p * 3)(gb[0].data_ptr(), gb[1].data_ptr(), gb[2].data_ptr())
    _lib.check(getattr(lib, name)(C.byref(f), C.byref(t), C.byref(p), int(segment), dq_p, dtw_p,
                                  db_p, df_p, g3, w.data_ptr(), w.numel(), _stream(stream)), name)
    if stream is not None:
        # temporaries freed here stay reserved until the caller's stream is done
        for x in (dq_t, dtw_t, db_t, df_t, w):
            if x is not None:
                x.record_stream(stream)
    return gb


def backward(B, grid, plane, params: Optional[Params] = None, segment: int = 32, dq=None, dtw=None,
             dend_b=None, dend_f=None, gb=None, stream=None, ws=None):
    """Reverse-mode derivative of the q2d map of (B, grid, plane) with respect to the
    field's node values (fastqsl_backward; a seed plane on a box face, or an interior one
    whose rotated-S0 lines are differentiated too). params.precision
    picks the form differentiated: all-FP64 (the default here), or F32X, whose FP32
    pass is replayed and reversed in FP32.

    dq, dtw: CUDA float64 tensors of nu*nv values (dL/dQ, dL/dTw), dend_b, dend_f:
    nu*nv x 3 (dL/d end points); any may be None. The result is ADDED into gb, a
    CUDA float64 tensor shaped like B (allocated as zeros if None), and returned.
    Lines are re-traced with checkpoints every `segment` accepted steps."""
    return _bwd_reverse("fastqsl_backward", B, grid, plane, params, segment, dq, dtw, dend_b,
                        dend_f, gb, stream, ws)


def q2d_record(B, grid, plane, params: Optional[Params] = None, segment: int = 32,
               want_lines: bool = False, stream=None, ws=None) -> dict:
    """The q2d map of (B, grid, plane) (all-FP64 unless params ask for F32X), traced
    once with the checkpoints of its derivative kept (fastqsl_q2d_record). The
    returned dict holds the map and,
    under "_ws", the workspace to hand to backward_recorded (which must not be
    written by anything else in between)."""
    lib, f, pl, p, need = _bwd_prepare(B, grid, plane, params, segment)
    w = _workspace(need, B.device, ws)
    m, s = _alloc_map(plane.nu * plane.nv, (plane.nv, plane.nu), B.device, want_lines)
    _lib.check(lib.fastqsl_q2d_record(C.byref(f), C.byref(pl), C.byref(p), int(segment), C.byref(s),
                                      w.data_ptr(), w.numel(), _stream(stream)), "fastqsl_q2d_record")
    m["_ws"] = w
    return m


def backward_recorded(B, grid, plane, rec: dict, params: Optional[Params] = None, segment: int = 32,
                      dq=None, dtw=None, dend_b=None, dend_f=None, gb=None, stream=None):
    """backward() of a map that q2d_record produced (same B, grid, plane, params and
    segment; rec: its result), without tracing the lines again (fastqsl_backward_recorded)."""
    return _bwd_reverse("fastqsl_backward_recorded", B, grid, plane, params, segment, dq, dtw,
                        dend_b, dend_f, gb, stream, rec["_ws"])


def q3d_backward(B, grid, voxels, params: Optional[Params] = None, segment: int = 32, dq=None,
                 dtw=None, dend_b=None, dend_f=None, gb=None, stream=None, ws=None):
    """backward() for the q3d map of (B, grid, voxels) (fastqsl_q3d_backward): dq, dtw
    hold nx*ny*nz values and dend_b, dend_f nx*ny*nz x 3, in map order (x fastest);
    the rotated-S0 voxels' extra lines are differentiated too (RKF45 only)."""
    return _bwd_reverse("fastqsl_q3d_backward", B, grid, voxels, params, segment, dq, dtw, dend_b,
                        dend_f, gb, stream, ws)


def q3d_record(B, grid, voxels, params: Optional[Params] = None, segment: int = 32,
               want_lines: bool = False, stream=None, ws=None) -> dict:
    """The q3d map of (B, grid, voxels), traced once with the checkpoints of its
    derivative kept (fastqsl_q3d_record); "_ws" holds the workspace for
    q3d_backward_recorded."""
    lib, f, v, p, need = _bwd_prepare(B, grid, voxels, params, segment)
    w = _workspace(need, B.device, ws)
    nx, ny, nz = (int(x) for x in voxels.n)
    m, s = _alloc_map(nx * ny * nz, (nz, ny, nx), B.device, want_lines)
    _lib.check(lib.fastqsl_q3d_record(C.byref(f), C.byref(v), C.byref(p), int(segment), C.byref(s),
                                      w.data_ptr(), w.numel(), _stream(stream)), "fastqsl_q3d_record")
    m["_ws"] = w
    return m


def q3d_backward_recorded(B, grid, voxels, rec: dict, params: Optional[Params] = None,
                          segment: int = 32, dq=None, dtw=None, dend_b=None, dend_f=None, gb=None,
                          stream=None):
    """q3d_backward() of a map that q3d_record produced, without tracing the lines
    again (fastqsl_q3d_backward_recorded)."""
    return _bwd_reverse("fastqsl_q3d_backward_recorded", B, grid, voxels, params, segment, dq, dtw,
                        dend_b, dend_f, gb, stream, rec["_ws"])
