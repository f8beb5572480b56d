"""Seeded synthetic inputs for LocalPower.

This package only draws inputs: the data matrix A with a controlled spectrum,
partition offsets, the Gaussian start matrix and the communication schedule.
No step of the method (local multiply, orthonormalisation, alignment,
aggregation, distance) is computed here, so the oracle and the HIP path can
both take their inputs from it without sharing any of the method's arithmetic.
"""

from .workloads import (  # noqa: F401
    Workload,
    haar,
    spectrum_c1,
    spectrum_gap,
    power_law_cov,
    lowrank_plus_noise,
    gaussian_rows,
    equal_offsets,
    lognormal_offsets,
    gaussian_start,
    fixed_schedule,
    decay_schedule,
    make_c1,
    make_c2,
    make_c3,
    make_c4,
    make_small,
)
