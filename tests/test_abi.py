"""The C-ABI library on the CPU: it loads, exports every entry point the header
declares, and its host logic (workspace queries, argument checks) works without a
GPU. No compute call is made here."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastqsl.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2208_12569_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2208_12569_amd import build

        build.build()
    return _lib.load()


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fastqsl_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ("fastqsl_trace", "fastqsl_q2d", "fastqsl_q3d", "fastqsl_backward"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2208_12569_amd import _lib

    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTS) == set(_declared())


def test_struct_sizes_match_header_layout(lib):
    from paper_2208_12569_amd import _lib

    # int64[3] + double[3] + double[3] + int32 + int32 + ptr[3]
    assert C.sizeof(_lib.fq_field) == 24 + 24 + 24 + 8 + 24 + 24
    assert C.sizeof(_lib.fq_params) == 5 * 8 + 8 + 4 * 4 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert C.sizeof(_lib.fq_plane) == 9 * 8 + 16 + 16
    assert C.sizeof(_lib.fq_voxels) == 9 * 8
    assert C.sizeof(_lib.fq_lines) == 10 * 8
    assert C.sizeof(_lib.fq_map) == 4 * 8 + 10 * 8 + 8 + 8


def _fake_field(n=(64, 64, 64), dtype=0):
    from paper_2208_12569_amd import _lib

    f = _lib.fq_field()
    f.n[:] = n
    f.origin[:] = (0.0, 0.0, 0.0)
    d = 1.0 / 63.0
    f.spacing[:] = (d, d, d)
    f.dtype = dtype
    for c in range(3):
        f.b[c] = 0x1000 * (c + 1)  # never dereferenced by the size query
    return f


def _plane(nu=128, z=0.0):
    from paper_2208_12569_amd import _lib

    p = _lib.fq_plane()
    p.origin[:] = (0.5 / nu, 0.5 / nu, z)
    p.u[:] = (1.0, 0.0, 0.0)
    p.v[:] = (0.0, 1.0, 0.0)
    p.nu = p.nv = nu
    p.du = p.dv = 1.0 / nu
    return p


def test_workspace_queries(lib):
    from paper_2208_12569_amd import _lib

    f = _fake_field()
    pl = _plane()
    p = _lib.fq_params()
    p.want_tw = 1
    n_on_face = lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p))
    assert n_on_face > 0
    nodes = 64 ** 3
    lines = 128 * 128
    # node records (16 + 8 bytes per node in FP32) + half-line records
    assert n_on_face >= nodes * 24 + 2 * lines * (24 + 8 + 8 + 1 + 2)
    # an interior plane adds the rotated-S0 buffers
    pl2 = _plane(z=0.5)
    n_inner = lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl2), 1, C.byref(p))
    assert n_inner > n_on_face
    # FP64 doubles the node records (and has no FP64 re-trace list)
    p.precision = _lib.FQ_PREC_F64
    n64 = lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p))
    assert n64 >= nodes * 48 + 2 * lines * (24 + 8 + 8 + 1 + 2)
    # the FP32 form without its FP64 pass needs no re-trace list
    p.precision = 0
    p.graze = -1.0
    assert lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p)) < n_on_face
    p.graze = 0.0
    # without Tw there are no curl records
    p.precision = 0
    p.want_tw = 0
    assert lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p)) < n_on_face
    v = _lib.fq_voxels()
    v.origin[:] = (0.01, 0.01, 0.01)
    v.spacing[:] = (0.02, 0.02, 0.02)
    v.n[:] = (8, 8, 8)
    assert lib.fastqsl_q3d_workspace_size(C.byref(f), C.byref(v), C.byref(p)) > 0
    assert lib.fastqsl_trace_workspace_size(C.byref(f), 100, C.byref(p)) > 0


def test_invalid_arguments_rejected_before_any_launch(lib):
    from paper_2208_12569_amd import _lib

    p = _lib.fq_params()
    pl = _plane()
    bad = _fake_field(n=(1, 64, 64))
    assert lib.fastqsl_q2d_workspace_size(C.byref(bad), C.byref(pl), 1, C.byref(p)) == 0
    f = _fake_field()
    f.spacing[1] = 0.0
    assert lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p)) == 0
    f = _fake_field()
    f.b[2] = None
    assert lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p)) == 0
    f = _fake_field()
    skew = _plane()
    skew.v[:] = (0.1, 1.0, 0.0)
    assert lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(skew), 1, C.byref(p)) == 0
    p.block = 100
    assert lib.fastqsl_q2d_workspace_size(C.byref(f), C.byref(pl), 1, C.byref(p)) == 0
    p.block = 0
    p.precision = 7
    m = _lib.fq_map()
    assert lib.fastqsl_q2d(C.byref(f), C.byref(pl), 1, C.byref(p), C.byref(m), None, 0,
                           None) == _lib.FQ_EINVAL
    p.precision = 0
    # null maps / workspace too small: rejected before anything is enqueued
    assert lib.fastqsl_q2d(C.byref(f), C.byref(pl), 1, C.byref(p), None, None, 0,
                           None) == _lib.FQ_EINVAL
    assert lib.fastqsl_q2d(C.byref(f), C.byref(pl), 1, C.byref(p), C.byref(m), C.c_void_p(256),
                           16, None) == _lib.FQ_ENOMEM
    assert lib.fastqsl_q2d(C.byref(f), C.byref(pl), 0, C.byref(p), C.byref(m), None, 0,
                           None) == _lib.FQ_EINVAL
    assert lib.fastqsl_strerror(_lib.FQ_ENOMEM) == b"workspace too small"


def test_interior_planes_in_a_batch_take_their_rotated_s0_room(lib):
    """A batch may mix interior and box-face planes; each interior plane adds its
    rotated-S0 room (four extra lines per point) to the workspace."""
    from paper_2208_12569_amd import _lib

    p = _lib.fq_params()
    fs = (_lib.fq_field * 2)(_fake_field(), _fake_field())
    face = lib.fastqsl_q2d_workspace_size(fs, (_lib.fq_plane * 2)(_plane(), _plane()), 2, C.byref(p))
    one = lib.fastqsl_q2d_workspace_size(fs, (_lib.fq_plane * 2)(_plane(z=0.5), _plane()), 2, C.byref(p))
    two = lib.fastqsl_q2d_workspace_size(fs, (_lib.fq_plane * 2)(_plane(z=0.5), _plane(z=0.25)), 2,
                                         C.byref(p))
    assert 0 < face < one < two


def test_python_layer_fails_loudly_without_gpu():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2208_12569_amd as fq

    with pytest.raises(RuntimeError, match="GPU"):
        fq.q2d(torch.zeros(3, 4, 4, 4), None, None)


def test_backward_workspace_query(lib):
    """The adjoint is taken on a seed plane (on a box face or interior), in either
    precision form and with Method I only; its workspace holds a pool of 2 +
    ceil(2048/segment) checkpoints of 64 bytes per half line."""
    from paper_2208_12569_amd import _lib

    f = _fake_field()
    pl = _plane(nu=64)
    p = _lib.fq_params()
    p.want_tw = 1
    p.precision = _lib.FQ_PREC_F32X
    assert lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(pl), C.byref(p), 32) > 0
    p.method = _lib.FQ_METHOD_II
    assert lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(pl), C.byref(p), 32) == 0
    p.method = _lib.FQ_METHOD_I
    p.precision = _lib.FQ_PREC_F64
    for seg in (0, -1, 5000):
        assert lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(pl), C.byref(p), seg) == 0
    n32 = lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(pl), C.byref(p), 32)
    # an interior plane also holds its rotated-S0 job's half lines (four lines per point)
    inner = _plane(nu=64, z=0.5)
    assert lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(inner), C.byref(p), 32) > n32
    halves = 2 * 64 * 64
    slots = 32768  # lanes of the reverse kernel, each with `segment` 48-byte step records
    assert n32 >= halves * (2048 // 32 + 2) * 64 + slots * 32 * 48
    n64 = lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(pl), C.byref(p), 64)
    assert n64 >= halves * (2048 // 64 + 2) * 64 + slots * 64 * 48
    p.max_steps = 1 << 40
    assert lib.fastqsl_backward_workspace_size(C.byref(f), C.byref(pl), C.byref(p), 32) == 0
    p.max_steps = 0
    # the call itself validates the gradient planes before touching the device
    gb = (C.c_void_p * 3)(None, None, None)
    rc = lib.fastqsl_backward(C.byref(f), C.byref(pl), C.byref(p), 32, None, None, None, None, gb,
                              None, 0, None)
    assert rc == _lib.FQ_EINVAL


def test_ctypes_layout_matches_compiled_header(tmp_path):
    """Every field of every struct of the header sits at the same offset in the
    binding's ctypes structs as in the C compiler's layout of the header."""
    import subprocess

    from paper_2208_12569_amd import _lib

    structs = {"fq_field": _lib.fq_field, "fq_params": _lib.fq_params, "fq_plane": _lib.fq_plane,
               "fq_voxels": _lib.fq_voxels, "fq_lines": _lib.fq_lines, "fq_map": _lib.fq_map}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fastqsl.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fld, _ in cls._fields_:
            lines.append(f'printf("{name} {fld} %zu\\n", offsetof({name}, {fld}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    seen = 0
    for row in out:
        if not row:
            continue
        name, fld, val = row.split()
        cls = structs[name]
        want = C.sizeof(cls) if fld == "size" else getattr(cls, fld).offset
        assert int(val) == want, (name, fld, int(val), want)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())
