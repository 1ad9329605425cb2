"""Seeded synthetic inputs shaped like the paper's workloads.

This package only *generates inputs*: station layouts, uvw tracks, channel
frequencies, flags, visibilities, A-terms and the taper.  It holds none of the
image-domain gridding arithmetic (no planning, no phasor sums, no transforms,
no adding), so both the FP64 oracle and the HIP path can consume the very same
arrays without sharing any of the method's code.
"""

from .workloads import (  # noqa: F401
    C0,
    Workload,
    make_workload,
    subset,
    WORKLOAD_NAMES,
)
from .taper import pswf_taper_1d, pswf_taper_2d  # noqa: F401
from .serving import serving_trace  # noqa: F401
