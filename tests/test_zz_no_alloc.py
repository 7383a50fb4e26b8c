"""fastqsl_q2d_static (the library's own device scratch, no workspace) against
fastqsl_q2d with a caller workspace, through the C-ABI: two calls in a row, the
second on a smaller input, equal bit for bit in both forms; a job too large for
the scratch is refused."""

import sys

import numpy as np
import pytest

import synth
from synth import Plane, cubic_grid

pytestmark = pytest.mark.gpu


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


def _same(a, b, label):
    for k in ("q", "tw", "length", "status"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x, y, equal_nan=True), (label, k)
    if "lines" in a:
        for k in ("end_b", "end_f", "face_b", "face_f"):
            assert np.array_equal(a["lines"][k].cpu().numpy(), b["lines"][k].cpu().numpy(),
                                  equal_nan=True), (label, k)


@pytest.mark.parametrize("prec", [0, 1], ids=["f32x", "f64"])
def test_static_scratch_equals_caller_workspace(fq, prec):
    import torch

    p = fq.Params(precision=prec)
    w = synth.config_c1(0)
    B = torch.from_numpy(w.field).cuda()
    big = [(B, w.grid, w.plane)]
    rng = np.random.default_rng(9)
    g = cubic_grid(40, 36, 30)
    pos, q = synth.draw_charges(rng, 6)
    Bs = torch.from_numpy(synth.charges_field(g, pos, q, dtype=np.float32)).cuda()
    small = [(Bs, g, Plane((0.013, 0.021, 0.0), (1, 0, 0), (0, 1, 0), 61, 45, 0.0161, 0.0211))]
    assert fq.q2d_workspace_size(big, p) <= fq.static_scratch_bytes()
    for label, jobs in (("c1 128x128", big), ("61x45 on 40x36x30", small)):
        _say(f"static scratch: {label}, precision {prec}")
        got = fq.q2d_static(jobs, p, want_lines=True)
        ref = fq.q2d_batch(jobs, p, want_lines=True)
        torch.cuda.synchronize()
        _same(got[0], ref[0], label)
        assert np.isfinite(got[0]["q"].cpu().numpy()).mean() > 0.9


def test_static_scratch_refuses_a_job_too_large(fq):
    import torch

    g = cubic_grid(256, 256, 160)
    B = torch.zeros((3, 160, 256, 256), dtype=torch.float32, device="cuda")
    jobs = [(B, g, synth.plane_z0(64))]
    assert fq.q2d_workspace_size(jobs) > fq.static_scratch_bytes()
    _say("static scratch: too large")
    with pytest.raises(RuntimeError, match="workspace too small"):
        fq.q2d_static(jobs)
