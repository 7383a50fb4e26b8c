"""The seeded input generators (CPU): the device-side charge-field generator
reproduces the NumPy one, and the batch draws are deterministic."""

import numpy as np
import torch

import synth
from synth.torch_fields import charges_field_torch


def test_torch_charges_field_equals_numpy():
    g = synth.cubic_grid(40, 33, 20)
    rng = np.random.default_rng(3)
    pos, q = synth.draw_charges(rng, 5)
    a = synth.charges_field(g, pos, q, dtype=np.float32)
    b = charges_field_torch(g, pos, q, torch.float32, "cpu", chunk=7).numpy()
    assert np.array_equal(a, b)
    a64 = synth.charges_field(g, pos, q)
    b64 = charges_field_torch(g, pos, q, torch.float64, "cpu").numpy()
    assert np.abs(a64 - b64).max() <= 1e-14 * np.abs(a64).max()


def test_torch_charges_field_gradient_is_the_unit_charge_field():
    g = synth.cubic_grid(9, 8, 7)
    pos = torch.tensor([[0.3, 0.4, -0.2], [0.6, 0.5, -0.3]], dtype=torch.float64)
    q = torch.tensor([1.0, -1.0], dtype=torch.float64, requires_grad=True)
    B = charges_field_torch(g, pos, q, torch.float64, "cpu")
    w = torch.randn(B.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
    (B * w).sum().backward()
    unit = synth.charges_field(g, pos[:1].numpy(), np.array([1.0]))
    assert abs(float(q.grad[0]) - float((unit * w.numpy()).sum())) < 1e-9


def test_c4_draws_are_deterministic():
    a = synth.fields.c4_specs(0)
    b = synth.fields.c4_specs(0)
    assert len(a) == 16
    for x, y in zip(a, b):
        assert x[0] == y[0] and x[1] == y[1] and x[4] == y[4]
        assert np.array_equal(x[2], y[2]) and np.array_equal(x[3], y[3])
        assert 64 <= x[1] <= 384 and x[4] in (128, 256, 512, 1024)
        assert 4 <= len(x[3]) <= 12 and abs(x[3].sum()) < 1e-12


def test_torch_tube_field_equals_numpy():
    from synth.torch_fields import tube_field_torch

    g = synth.cubic_grid(41, 37, 23)
    qt = synth.fields.tube_q_for_turns(0.2, -0.08, 1.5)
    for n, c in ((1, (0.5, 0.35, -0.08)), (0, (0.65, 0.5, -0.08))):
        a = synth.fields.tube_field(g, c, 0.2, 0.08, 1.0, qt, plane_normal=n, chunk=5)
        b = tube_field_torch(g, c, 0.2, 0.08, 1.0, qt, n, "cpu", chunk=6).numpy()
        assert np.abs(a - b).max() <= 1e-14 * max(np.abs(a).max(), 1.0)
        assert np.array_equal(a.astype(np.float32), b.astype(np.float32))
