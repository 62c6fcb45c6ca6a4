"""MI355X-native FFT beam-propagation z-march (two-beam Bragg diffraction in
deformed crystals, time-dependent via independent frequency slices).

The compute path is libbpm.so (hand-written HIP for gfx950, C ABI declared in
include/bpm.h); this package is its thin Python binding.
"""

from ._native import (  # noqa: F401
    Batch,
    BpmError,
    Job,
    Plan,
    Plan3D,
    propagate_batch,
    PRECISION,
    LIB_PATH,
    lib,
    last_error,
)
