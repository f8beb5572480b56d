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
    spectrum_cluster,
    power_law_cov,
    lowrank_plus_noise,
    gaussian_rows,
    equal_offsets,
    lognormal_offsets,
    gaussian_start,
    fixed_schedule,
    decay_schedule,
    make_fp64_2000x100,
    make_fp32_262144x1024,
    make_bf16_1048576x2048,
    make_fp32_uneven_500000x4096,
    make_small,
)
