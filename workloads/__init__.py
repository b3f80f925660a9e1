"""Seeded synthetic inputs for the free-flight expansion workloads.

This package holds only the generators of initial fields and the problem
parameters of each workload. It contains none of the expansion arithmetic, so
both the CPU oracle and the GPU path can draw their inputs from it without
sharing any of the method's code.
"""

from .generators import (  # noqa: F401
    C4_SHAPES,
    c4_fields_c64,
    WORKLOADS,
    centred_coords,
    random_field,
    Workload,
    gaussian_random_field,
    make_c1,
    make_c2,
    make_c3,
    make_c4,
    make_c5,
    make_workload,
    soliton_gaussian_1d,
    thomas_fermi_phase_2d,
    two_cloud_3d,
    ensemble_member_3d,
)
