"""MI355X (gfx950) HOQRI: higher-order QR iteration for sparse Tucker decomposition.

The computation runs in libhoqri.so (HIP kernels behind the C ABI of
include/hoqri.h); this package is its thin Python binding.
"""
from ._lib import (  # noqa: F401
    Arena,
    HoqriError,
    ServeResult,
    Server,
    Plan,
    Stats,
    hoqri_core,
    hoqri_orth,
    hoqri_orth_workspace_size,
    hoqri_plan_create,
    hoqri_plan_info,
    hoqri_plan_workspace_size,
    hoqri_run,
    hoqri_sketch_start,
    hoqri_status_string,
    hoqri_timing_enable,
    hoqri_timing_read,
    hoqri_ttmctc,
)
