"""gfx950-native multi-stixel segmentation (Hernandez-Juarez et al.,
"GPU-accelerated real-time stixel computation").

The work runs in hand-written HIP kernels behind the C ABI of
``include/stixels.h``; this package is the argument-marshalling binding.
"""

from .binding import (  # noqa: F401
    EXPORTS,
    Batch,
    FrameOutput,
    Sgm,
    Stixels,
    StixelsError,
    compute_batch,
    decode_records,
    host_table,
    lib,
    selftest_mean,
    status_string,
)

__all__ = ["Batch", "Sgm", "Stixels", "FrameOutput", "StixelsError", "compute_batch", "decode_records",
           "host_table", "lib", "selftest_mean", "status_string", "EXPORTS"]
