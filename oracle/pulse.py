"""Time <-> frequency transform of a pulse (Eq. tdp) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module; the product library never does.

Section 3 (time-dependent problems) turns a pulse into independent
stationary problems: the incident field is Fourier transformed along t, each
frequency is marched on its own, and the outputs are transformed back.  This
module writes that pair out as its definition, an explicit sum over the grid
points, with the phase of every term reduced exactly in integer arithmetic.

Readings (the paper prints the pair without fixing the grids or the factor
of the inverse):
  - centred grids: t_i = (i - N/2) dt and Omega_j = (j - N/2) dOmega with
    dOmega = 2 pi / (N dt), i, j = 0..N-1 (the discrete Fourier pair);
    Omega is the offset from the carrier omega_0 = 2 pi c / lambda, so slice
    j has the relative detuning delta_j = Omega_j / omega_0;
  - forward, the printed sign: psi(Omega_j) = dt sum_i psi(t_i) exp(+i Omega_j t_i);
  - inverse: psi(t_i) = (dOmega / 2 pi) sum_j psi(Omega_j) exp(-i Omega_j t_i);
    the printed inverse carries d omega alone, which makes the round trip
    2 pi times the identity; the 1/(2 pi) is taken so that it is the identity.
"""

from __future__ import annotations

import numpy as np

__all__ = ["C_LIGHT", "time_grid", "frequency_grid", "detuning",
           "to_frequency", "to_time"]

C_LIGHT = 299792458.0   # m/s


def time_grid(N: int, dt: float) -> np.ndarray:
    """t_i = (i - N/2) dt."""
    return (np.arange(N) - N // 2) * float(dt)


def frequency_grid(N: int, dt: float) -> np.ndarray:
    """Omega_j = (j - N/2) 2 pi / (N dt) (offsets from the carrier)."""
    return (np.arange(N) - N // 2) * (2.0 * np.pi / (N * float(dt)))


def detuning(N: int, dt: float, lam: float) -> np.ndarray:
    """delta_j = Omega_j / omega_0 with omega_0 = 2 pi c / lambda."""
    return frequency_grid(N, dt) / (2.0 * np.pi * C_LIGHT / float(lam))


def _phase(N: int, sign: int) -> np.ndarray:
    """exp(sign i Omega_j t_i) for all (j, i): Omega_j t_i = 2 pi m / N with
    m = (j - N/2)(i - N/2), reduced mod N exactly in integers."""
    k = np.arange(N, dtype=np.int64) - N // 2
    m = np.mod(np.outer(k, k), N)
    return np.exp(sign * 2j * np.pi * m / N)


def to_frequency(field_t, dt: float) -> np.ndarray:
    """psi(Omega_j, x) = dt sum_i psi(t_i, x) exp(+i Omega_j t_i), for a field
    laid out [N][Nx] (time first)."""
    f = np.asarray(field_t, dtype=np.complex128)
    N = f.shape[0]
    return float(dt) * (_phase(N, +1) @ f)


def to_time(field_w, dt: float) -> np.ndarray:
    """psi(t_i, x) = (dOmega / 2 pi) sum_j psi(Omega_j, x) exp(-i Omega_j t_i),
    dOmega / 2 pi = 1 / (N dt), for a field laid out [N][Nx]."""
    f = np.asarray(field_w, dtype=np.complex128)
    N = f.shape[0]
    # _phase is symmetric in (j, i)
    return (_phase(N, -1) @ f) / (N * float(dt))
