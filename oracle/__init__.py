"""CPU oracle of the FFT beam-propagation z-march -- TEST INFRASTRUCTURE.

This package is the slow, obviously correct FP64 reference that the GPU path
is checked against.  It shares no code with the GPU library and never imports
it.  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import, call or execute anything in here; the product path must never route
through it.

Pinning: every function here is checked by the CPU test suite against
quantities fixed independently of this code (closed forms, invariants,
brute-force transforms, textbook dynamical theory); see tests/test_oracle_*.py.
"""

from .bpm import (  # noqa: F401
    TWO_PI_X,
    Problem,
    beam_constants,
    slice_constants,
    coupling_constants,
    wavenumbers,
    propagator,
    crystal_mask,
    deformation_factor,
    split_coefficients,
    march,
)
from .bpm3d import (  # noqa: F401
    Problem3D,
    wavenumbers_y,
    propagator3d,
    crystal_mask3d,
    march3d,
)
