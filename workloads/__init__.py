"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This package only *draws* inputs: sparse SPD matrices in CSR form, right-hand
sides, grid coordinates and partition target weights.  It contains none of the
solver's arithmetic (no partitioning, no SpMV, no CG); both the HIP library and
the CPU oracle consume what it produces.

The matrices stand in for the finite-element / finite-difference SPD systems the
paper solves (model problem -Laplace(u) = f with homogeneous Dirichlet data,
Section 3.4, and the engineering matrices of the experiments section).
"""
from .generators import (  # noqa: F401
    CSR,
    Workload,
    poisson2d,
    poisson3d,
    diffusion2d_lognormal,
    diffusion3d_lognormal,
    diffusion3d_grf,
    q1hex_lognormal,
    batch2d_lognormal,
    random_spd_csr,
    uniform_rhs,
    rcb_weights,
    grid_coords,
    config,
    CONFIG_NAMES,
)
