"""MI355X-native LocalPower: HIP kernels for gfx950 behind a C ABI (include/lp.h).

The Python layer is a thin ctypes binding (same names as the C entry points);
PyTorch supplies device memory and streams only.
"""

from ._lib import (  # noqa: F401
    LPError,
    LP_OK,
    LP_ENOTCONV,
    Problem,
    Server,
    load,
    lp_workspace_size,
    lp_create,
    lp_destroy,
    lp_set_tuning,
    lp_get_tuning,
    lp_autotune,
    lp_run,
    lp_solve,
    lp_gram_bytes,
    lp_gram_enable,
    lp_gram_disable,
    lp_eta,
    lp_local_multiply,
    lp_profile_local_multiply,
    lp_orth,
    lp_orth_noalloc,
    lp_align,
    lp_sin_theta,
    lp_generate,
    lp_bandwidth_probe,
    lp_copy_probe,
)
