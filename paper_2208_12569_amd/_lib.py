"""ctypes view of libfastqsl.so: the structs and entry points of include/fastqsl.h.

Loading fails loudly if the library has not been built: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastqsl.so")

FQ_OK = 0
FQ_EINVAL = -1
FQ_ENOMEM = -2
FQ_EHIP = -3
FQ_EUNSUPPORTED = -4

FQ_DT_F32 = 0
FQ_DT_F64 = 1
FQ_PREC_F32X = 0
FQ_PREC_F64 = 1
FQ_SCHEME_RKF45 = 0
FQ_SCHEME_RK4 = 1
FQ_SCHEME_RK4_38 = 2
FQ_METHOD_I = 0
FQ_METHOD_II = 1

ST_OK = 0
ST_OUTSIDE = 1
ST_NULLB = 2
ST_MAXSTEPS = 4
ST_NONFINITE = 8
ST_ONESIDED = 16
ST_MIXEDFACE = 32
ST_EDGE = 64
ST_ROTATED = 128
ST_NOTAPE = 256
ST_FATAL = ST_OUTSIDE | ST_NULLB | ST_MAXSTEPS | ST_NONFINITE


class fq_field(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("dtype", C.c_int32), ("reserved", C.c_int32), ("b", C.c_void_p * 3),
                ("coord", C.c_void_p * 3)]


class fq_params(C.Structure):
    _fields_ = [("tol_perp", C.c_double), ("step_perp", C.c_double), ("step_min", C.c_double),
                ("tol_floor", C.c_double), ("edge_eps", C.c_double), ("max_steps", C.c_int64),
                ("precision", C.c_int32), ("want_tw", C.c_int32), ("block", C.c_int32),
                ("waves_per_cu", C.c_int32), ("graze", C.c_double), ("stats", C.c_void_p),
                ("events", C.c_void_p), ("qfix", C.c_double), ("tape_steps", C.c_int64),
                ("scheme", C.c_int32), ("method", C.c_int32), ("in_flight", C.c_int32),
                ("reserved2", C.c_int32)]


class fq_plane(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("u", C.c_double * 3), ("v", C.c_double * 3),
                ("nu", C.c_int64), ("nv", C.c_int64), ("du", C.c_double), ("dv", C.c_double)]


class fq_voxels(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("spacing", C.c_double * 3), ("n", C.c_int64 * 3)]


class fq_cylinder(C.Structure):
    _fields_ = [("centre", C.c_double * 2), ("radius", C.c_double), ("theta0", C.c_double),
                ("dtheta", C.c_double), ("ntheta", C.c_int64), ("z0", C.c_double),
                ("dz", C.c_double), ("nz", C.c_int64)]


FQ_FACE_CYL = 6


class fq_lines(C.Structure):
    _fields_ = [("end_b", C.c_void_p), ("end_f", C.c_void_p), ("face_b", C.c_void_p),
                ("face_f", C.c_void_p), ("bn_b", C.c_void_p), ("bn_f", C.c_void_p),
                ("bn0", C.c_void_p), ("tw", C.c_void_p), ("length", C.c_void_p),
                ("status", C.c_void_p)]


class fq_map(C.Structure):
    _fields_ = [("q", C.c_void_p), ("tw", C.c_void_p), ("length", C.c_void_p),
                ("status", C.c_void_p), ("lines", fq_lines), ("qperp", C.c_void_p),
                ("fledge", C.c_void_p)]


EXPORTS = [
    "fastqsl_trace_workspace_size", "fastqsl_trace",
    "fastqsl_q2d_workspace_size", "fastqsl_q2d",
    "fastqsl_q3d_workspace_size", "fastqsl_q3d",
    "fastqsl_qcyl_workspace_size", "fastqsl_qcyl",
    "fastqsl_backward_workspace_size", "fastqsl_backward",
    "fastqsl_q2d_record", "fastqsl_backward_recorded",
    "fastqsl_q3d_backward_workspace_size", "fastqsl_q3d_backward",
    "fastqsl_q3d_record", "fastqsl_q3d_backward_recorded",
    "fastqsl_strerror", "fastqsl_version",
    "fastqsl_static_scratch_bytes", "fastqsl_q2d_static",
]

_lib = None


def load():
    """Load libfastqsl.so (built in-tree by paper_2208_12569_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library then binds to the HIP runtime torch has loaded (both
    # carry the soname libamdhip64.so.7), so torch's streams are valid handles here
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2208_12569_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.fastqsl_trace_workspace_size.argtypes = [P(fq_field), C.c_int64, P(fq_params)]
    lib.fastqsl_trace_workspace_size.restype = C.c_size_t
    lib.fastqsl_trace.argtypes = [P(fq_field), C.c_void_p, C.c_int64, C.c_void_p, P(fq_params),
                                  P(fq_lines), C.c_void_p, C.c_size_t, C.c_void_p]
    lib.fastqsl_trace.restype = C.c_int
    lib.fastqsl_q2d_workspace_size.argtypes = [P(fq_field), P(fq_plane), C.c_int, P(fq_params)]
    lib.fastqsl_q2d_workspace_size.restype = C.c_size_t
    lib.fastqsl_q2d.argtypes = [P(fq_field), P(fq_plane), C.c_int, P(fq_params), P(fq_map),
                                C.c_void_p, C.c_size_t, C.c_void_p]
    lib.fastqsl_q2d.restype = C.c_int
    lib.fastqsl_q3d_workspace_size.argtypes = [P(fq_field), P(fq_voxels), P(fq_params)]
    lib.fastqsl_q3d_workspace_size.restype = C.c_size_t
    lib.fastqsl_q3d.argtypes = [P(fq_field), P(fq_voxels), P(fq_params), P(fq_map), C.c_void_p,
                                C.c_size_t, C.c_void_p]
    lib.fastqsl_q3d.restype = C.c_int
    lib.fastqsl_qcyl_workspace_size.argtypes = [P(fq_field), P(fq_cylinder), P(fq_params)]
    lib.fastqsl_qcyl_workspace_size.restype = C.c_size_t
    lib.fastqsl_qcyl.argtypes = [P(fq_field), P(fq_cylinder), P(fq_params), P(fq_map), C.c_void_p,
                                 C.c_size_t, C.c_void_p]
    lib.fastqsl_qcyl.restype = C.c_int
    lib.fastqsl_backward_workspace_size.argtypes = [P(fq_field), P(fq_plane), P(fq_params),
                                                    C.c_int]
    lib.fastqsl_backward_workspace_size.restype = C.c_size_t
    lib.fastqsl_backward.argtypes = [P(fq_field), P(fq_plane), P(fq_params), C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p * 3, C.c_void_p, C.c_size_t, C.c_void_p]
    lib.fastqsl_backward.restype = C.c_int
    lib.fastqsl_q2d_record.argtypes = [P(fq_field), P(fq_plane), P(fq_params), C.c_int, P(fq_map),
                                       C.c_void_p, C.c_size_t, C.c_void_p]
    lib.fastqsl_q2d_record.restype = C.c_int
    lib.fastqsl_backward_recorded.argtypes = lib.fastqsl_backward.argtypes
    lib.fastqsl_backward_recorded.restype = C.c_int
    lib.fastqsl_q3d_backward_workspace_size.argtypes = [P(fq_field), P(fq_voxels), P(fq_params),
                                                        C.c_int]
    lib.fastqsl_q3d_backward_workspace_size.restype = C.c_size_t
    lib.fastqsl_q3d_backward.argtypes = [P(fq_field), P(fq_voxels)] + lib.fastqsl_backward.argtypes[2:]
    lib.fastqsl_q3d_backward.restype = C.c_int
    lib.fastqsl_q3d_record.argtypes = [P(fq_field), P(fq_voxels)] + lib.fastqsl_q2d_record.argtypes[2:]
    lib.fastqsl_q3d_record.restype = C.c_int
    lib.fastqsl_q3d_backward_recorded.argtypes = lib.fastqsl_q3d_backward.argtypes
    lib.fastqsl_q3d_backward_recorded.restype = C.c_int
    lib.fastqsl_static_scratch_bytes.argtypes = []
    lib.fastqsl_static_scratch_bytes.restype = C.c_size_t
    lib.fastqsl_q2d_static.argtypes = [P(fq_field), P(fq_plane), C.c_int, P(fq_params), P(fq_map),
                                       C.c_void_p]
    lib.fastqsl_q2d_static.restype = C.c_int
    lib.fastqsl_strerror.argtypes = [C.c_int]
    lib.fastqsl_strerror.restype = C.c_char_p
    lib.fastqsl_version.argtypes = []
    lib.fastqsl_version.restype = C.c_char_p
    _lib = lib
    return lib


def check(rc: int, what: str):
    if rc != FQ_OK:
        msg = load().fastqsl_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} ({rc})")
