"""Seeded synthetic workloads: voxel grids, point-dipole coil geometries and
random current / field vectors.

This package holds geometry and random numbers only.  It evaluates no field,
compresses nothing and multiplies no matrices, so that both the CPU reference
(``oracle/``) and the GPU library draw their inputs from it without sharing any
of the method's arithmetic.
"""
from .configs import (  # noqa: F401
    BODYCOIL, C0, FREQ_3T, aca_rank, FREQ_7T, Grid, Workload, complex_normal, make,
    make_batch, make_bodycoil, NAMES,
)
