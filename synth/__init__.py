"""Seeded synthetic input generators for the induction-log integral-equation solver.

This package only builds inputs: voxel grids, per-cell conductivity tensors,
transmitters and sub-domain partitions.  It holds none of the solver's
arithmetic (no Green's tensor, no background field, no FFT, no Krylov step), so
both the CPU oracle and the GPU path may take their inputs from it.
"""
from .models import (  # noqa: F401
    Problem,
    cell_centres,
    ti_tensor6,
    config0,
    config1,
    config2,
    config3,
    config4_train,
    config4_eval,
    example1,
    random_problem,
    tensor6_to_3x3,
    default_origin,
)
