"""Seeded synthetic inputs for the FFT beam-propagation z-march.

This package is shared by the oracle, the tests and the benchmark.  It builds
problem parameters, incident boundary fields and displacement fields; it holds
none of the propagation arithmetic (no FFT, no propagator, no coupling).
"""

from .configs import (  # noqa: F401
    Workload,
    small,
    c1_perfect_crystal,
    c2_bent_crystal,
    c3_thermal_bump,
    c4_problem_specs,
    c4_problem,
    c5_request_trace,
    darwin_relative_width,
    detuning_grid,
    pulse_field,
    by_name,
    Workload3D,
    small3d,
    heat_bump_3d,
)
