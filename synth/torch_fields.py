"""Device-side generators for the larger synthetic cubes.

The same point-charge fields as ``fields.charges_field`` and flux tubes as
``fields.tube_field``, evaluated with torch on the GPU (float64 arithmetic, rounded
once to the output type), so that big batches and cubes are generated in seconds and a field model can be differentiated with respect to its
charge positions and strengths. Input generation only: nothing here traces lines or
forms Q.
"""

from __future__ import annotations

from typing import List

import torch

from .fields import Grid, Workload, c3_spec, c4_specs, cubic_grid, plane_z0


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


def tube_field_torch(grid: Grid, center, R0: float, a: float, B0: float, q: float,
                     plane_normal: int = 1, device="cuda", chunk: int = 32) -> torch.Tensor:
    """fields.tube_field (the arched, uniformly twisted torus-sector tube) evaluated
    with torch in float64, shape (3, nz, ny, nx)."""
    ax = [torch.arange(n, dtype=torch.float64, device=device) * d + o
          for o, n, d in zip(grid.origin, (grid.nx, grid.ny, grid.nz), grid.spacing)]
    out = torch.zeros((3,) + tuple(grid.shape), dtype=torch.float64, device=device)
    cx, cy, cz = center
    n = plane_normal
    ip = 0 if n == 1 else 1
    for k0 in range(0, grid.nz, chunk):
        zz = ax[2][k0:k0 + chunk].view(-1, 1, 1)
        yy = ax[1].view(1, -1, 1)
        xx = ax[0].view(1, 1, -1)
        zz, yy, xx = torch.broadcast_tensors(zz, yy, xx)
        h = (xx - cx) if ip == 0 else (yy - cy)
        w = zz - cz
        R = torch.sqrt(h * h + w * w)
        R = torch.where(R > 1e-300, R, torch.full_like(R, 1e-300))
        eRh, eRw = h / R, w / R
        ephh, ephw = -eRw, eRh
        eta = (yy - cy) if n == 1 else (xx - cx)
        xi = R - R0
        rho = torch.sqrt(xi * xi + eta * eta)
        s = torch.clamp(1.0 - (rho / a) ** 2, min=0.0)
        f = s * s * s
        amp = B0 * (R0 / R) * f
        bh = amp * (ephh + q * (-eta) * eRh)
        bw = amp * (ephw + q * (-eta) * eRw)
        bn = amp * (q * xi)
        comp_h = 0 if ip == 0 else 1
        k1 = k0 + zz.shape[0]
        out[comp_h, k0:k1] += bh
        out[2, k0:k1] += bw
        out[n, k0:k1] += bn
    return out


def config_c3_torch(seed: int = 0, nvox=(256, 256, 128), device="cuda") -> Workload:
    """config_c3's cube generated on the device (field = float32 tensor), with the
    same roundings: the charge field and each tube rounded to float32 separately and
    summed in float32."""
    g, pos, q, tubes, vox, qt = c3_spec(seed, nvox)
    with torch.no_grad():
        B = charges_field_torch(g, pos, q, torch.float32, device)
        for c, R0, a, B0, qq, n in tubes:
            B += tube_field_torch(g, c, R0, a, B0, qq, n, device).to(torch.float32)
    return Workload("c3_charges10_tubes2_512x512x256", g, B, voxels=vox,
                    meta={"charges": (pos, q), "tube_q": qt})
