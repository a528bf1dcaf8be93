"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only builds meshes and per-face subdomain labels.  It holds none of
the parameterization arithmetic, so both the CPU oracle and the GPU path may use
it without sharing any of the method's code.
"""
from .meshes import (  # noqa: F401
    SEED_BASE,
    MeshCase,
    grid_mesh,
    block_labels,
    bump_field,
    case_c1,
    case_c2,
    case_c3,
    case_c5,
    small_grid_case,
    small_sphere_case,
    icosphere,
    guillotine_labels,
    c4_training_meshes,
)
