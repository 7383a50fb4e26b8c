"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package produces magnetic-field cubes and seed specifications only. It holds
none of the tracing, twist or squashing-factor arithmetic: those live separately in
the CPU oracle (``oracle/``) and in the HIP library (``paper_2208_12569_amd/``).
"""

from .fields import (  # noqa: F401
    Grid,
    Plane,
    Cylinder,
    Voxels,
    cubic_grid,
    geometric_axis,
    clustered_axis,
    stretched_grid,
    draw_charges,
    charges_field,
    tube_field,
    linear_field,
    quadrupole_field,
    plane_z0,
    config_c1,
    config_c1s,
    config_c2s,
    config_c2,
    config_c3,
    config_c4,
    config_c5,
)
