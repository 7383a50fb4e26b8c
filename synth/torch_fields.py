"""Device-side generators for the larger synthetic cubes.

The same point-charge fields as ``fields.charges_field``, evaluated with torch on the
GPU (float64 arithmetic, rounded once to the output type), so that big batches are
generated in seconds and a field model can be differentiated with respect to its
charge positions and strengths. Input generation only: nothing here traces lines or
forms Q.
"""

from __future__ import annotations

from typing import List

import torch

from .fields import Grid, Workload, c4_specs, cubic_grid, plane_z0


def charges_field_torch(grid: Grid, pos, q, dtype=torch.float32, device="cuda",
                        chunk: int = 32) -> torch.Tensor:
    """B(r) = sum_i q_i (r - r_i) / |r - r_i|^3 at every node, shape (3, nz, ny, nx).

    pos (n, 3) and q (n,) may be tensors that require grad; the result is then
    differentiable with respect to them."""
    pos = torch.as_tensor(pos, dtype=torch.float64, device=device)
    q = torch.as_tensor(q, dtype=torch.float64, device=device)
    ax = [torch.arange(n, dtype=torch.float64, device=device) * d + o
          for o, n, d in zip(grid.origin, (grid.nx, grid.ny, grid.nz), grid.spacing)]
    x = ax[0].view(1, 1, -1)
    y = ax[1].view(1, -1, 1)
    parts = []
    for k0 in range(0, grid.nz, chunk):
        z = ax[2][k0:k0 + chunk].view(-1, 1, 1)
        acc = None
        for i in range(pos.shape[0]):
            dx = x - pos[i, 0]
            dy = y - pos[i, 1]
            dz = z - pos[i, 2]
            r2 = dx * dx + dy * dy + dz * dz
            f = q[i] / (r2 * torch.sqrt(r2))
            term = torch.stack(torch.broadcast_tensors(f * dx, f * dy, f * dz))
            acc = term if acc is None else acc + term
        parts.append(acc.to(dtype))
    return torch.cat(parts, dim=1).contiguous()


def config_c4_torch(seed: int = 0, device="cuda", **kw) -> List[Workload]:
    """config_c4's batch with the fields generated on the device (field = tensor)."""
    jobs = []
    for name, E, pos, q, side in c4_specs(seed, **kw):
        g = cubic_grid(E, E, E)
        with torch.no_grad():
            B = charges_field_torch(g, pos, q, torch.float32, device)
        jobs.append(Workload(name, g, B, plane=plane_z0(side), meta={"charges": (pos, q)}))
    return jobs
