"""Image Domain Gridding on MI355X (gfx950): HIP kernels behind a C ABI.

The hot path -- subgrid planning, the per-subgrid image-domain phasor sum with
A-terms and taper, the subgrid transform, the adder, and the reverse chain --
lives in libidg.so (C ABI in include/idg.h).  This package is its thin Python
binding; device arrays are torch tensors, used only for memory and streams.
"""

from ._lib import (  # noqa: F401
    IDG_PHASE_FP32,
    IDG_STRICT,
    IDGError,
    LIB_PATH,
    NOALLOC_SCRATCH_BYTES,
    Plan,
    SUBGRID_FIELDS,
    add_subgrids,
    degrid,
    grid,
    grid_noalloc,
    grid_subgrids,
    grid_to_image,
    image_to_grid,
    optimal_taper,
    taper_shift_for_plan,
    wstack_to_image,
    image_to_wstack,
    taper_correction,
    lib,
    profile,
    profile_read,
    device_rates,
    trim_scratch,
    split_subgrids,
    subgrid_fft,
    sync,
    version,
)
