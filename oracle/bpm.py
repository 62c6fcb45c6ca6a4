"""Plain CPU oracle of the two-beam FFT BPM z-march (FP64).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product library never does.

It follows the paper step by step, with no blocking, fusion or reordering:

  * Eq. fov4  -- one split step: FFT along x, multiply by the free-propagation
    phase, inverse FFT, then the real-space susceptibility factor.
  * Eq. fov7  -- two slowly varying envelopes a = psi~_+ (carrier +h/2) and
    b = psi~_- (carrier -h/2).
  * Eq. fov10 -- the coupled step: a' = a_p d0 + b_p d'_{+1},
    b' = b_p d0 + a_p d'_{-1}, where x_p is x after free propagation.
  * Eqs. fov8, fov9, fov11, fov12 -- d0 and d_{+-1} are the n = 0, +-1
    Fourier coefficients (Jacobi-Anger) of exp(i dZ (chi0 + chih e^{ihx}
    + chihbar e^{-ihx}) / (2 cos alpha)), times the crystal mask.
  * Eq. Authier -- deformation: d'_{n} = d_n exp(i n h u(x, z)).
  * Zassenhaus-like factor (Section 2.1, end): d0 -> d0 exp(D2 dZ^2 / 2).
  * Eq. split-op -- optional 2nd / 4th order products of A and B.
  * Eq. tdp -- a pulse is a stack of independent frequency slices.

Readings taken where the paper is silent or garbled (each is listed with its
reason in the design notes):
  - physical Fourier convention: a component exp(+iKx) of psi~_+ propagates
    with kz = sqrt(k^2 - (K + h/2)^2), of psi~_- with sqrt(k^2 - (K - h/2)^2);
  - the per-step operators use the step length dZ = k dz (not z);
  - the full kz is kept in the free-propagation phase (Eq. fov4 as printed);
  - chih != chihbar is handled by the generating function of exp(a t + b/t):
    d0 = J0(sqrt(q)) g0, d_{+1} = i dZ chih/(2c) * 2J1(sqrt(q))/sqrt(q) * g0,
    d_{-1} the same with chihbar, q = dZ^2 chih chihbar / c^2,
    g0 = exp(i dZ chi0 / (2c)); D2 dZ^2/2 generalises to q/8;
  - cos(alpha) per slice is c = sqrt(1 - (h / 2k)^2);
  - within a step: propagate first, then couple with u and the mask taken at
    the step's start z_n = n dz;
  - the sign of the deformation phase is the printed exp(+i n h.u);
  - periodic transverse window (plain FFT, no absorbing layer).

Precision: fields and all step arithmetic are float64 / complex128.  The
propagator phase dz*kz (about 2.5e4 rad at the default workload) is evaluated
and reduced modulo 2*pi in x87 extended precision before rounding to float64,
so that the per-step phase carries only float64 rounding (~1e-16 rad) and not
the ~1e-12 rad that a float64 evaluation of a 2.5e4 rad phase would repeat
every step.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import special

__all__ = [
    "TWO_PI_X", "Problem", "beam_constants", "slice_constants",
    "coupling_constants", "wavenumbers", "propagator", "crystal_mask",
    "deformation_factor", "split_coefficients", "march",
]

# 2*pi in x87 extended precision (64-bit significand).
TWO_PI_X = np.arctan(np.longdouble(1)) * 8


class Problem:
    """Parameters of one problem (all slices share them except delta)."""

    def __init__(self, Nx, dx, dz, Nz, chi0, chih, chihbar, theta_B, lam,
                 delta, x_front=0.0, thickness=math.inf, zassenhaus=True,
                 split_order=1, mask=None):
        self.Nx = int(Nx)
        self.dx = float(dx)
        self.dz = float(dz)
        self.Nz = int(Nz)
        self.chi0 = complex(chi0)
        self.chih = complex(chih)
        self.chihbar = complex(chihbar)
        self.theta_B = float(theta_B)
        self.lam = float(lam)
        self.delta = np.atleast_1d(np.asarray(delta, dtype=np.float64))
        self.x_front = float(x_front)
        self.thickness = float(thickness)
        self.zassenhaus = bool(zassenhaus)
        self.split_order = int(split_order)
        # optional general crystal mask Pi[n][j] (bool, Nz x Nx) replacing
        # the slab: any crystal shape in the (x, z) plane
        self.mask = None if mask is None else np.asarray(mask, dtype=bool).reshape(Nz, Nx)

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(Nx=w.Nx, dx=w.dx, dz=w.dz, Nz=w.Nz, chi0=w.chi0, chih=w.chih,
                  chihbar=w.chihbar, theta_B=w.theta_B, lam=w.lam,
                  delta=w.delta, x_front=w.x_front, thickness=w.thickness)
        kw.update(over)
        return cls(**kw)

    @property
    def Nomega(self):
        return len(self.delta)


def beam_constants(p: Problem):
    """k0 = 2 pi / lambda and the reciprocal-lattice vector h = 2 k0 sin(theta_B)
    (Bragg's law), in float64."""
    k0 = 2.0 * math.pi / p.lam
    h = 2.0 * k0 * math.sin(p.theta_B)
    return k0, h


def slice_constants(p: Problem, delta: float):
    """Per-slice wavenumber k = k0 (1 + delta), cos(alpha) = sqrt(1 - (h/2k)^2)
    (the mean propagation direction of the two bands) and dZ = k dz."""
    k0, h = beam_constants(p)
    k = k0 * (1.0 + delta)
    s = 0.5 * h / k
    c = math.sqrt(1.0 - s * s)
    return k, c, k * p.dz


def coupling_constants(p: Problem, delta: float, frac: float = 1.0):
    """(d0, d_{+1}, d_{-1}) of one slice for a B sub-step of length frac*dz.

    Jacobi-Anger coefficients of exp(i dZ delta_eps / (2c)) with
    delta_eps = chi0 + chih e^{ihx} + chihbar e^{-ihx}; the generating function
    gives d0 = J0(sqrt(q)) g0 and d_{+-1} = (i dZ chi_{h/hbar} / 2c)
    * 2 J1(sqrt(q))/sqrt(q) * g0 (both even in sqrt(q), so branch-free);
    the Zassenhaus-like factor multiplies d0 by exp(q/8)."""
    _, c, dZ = slice_constants(p, delta)
    dZ = frac * dZ
    q = dZ * dZ * p.chih * p.chihbar / (c * c)
    g0 = np.exp(1j * dZ * p.chi0 / (2.0 * c))
    z = np.sqrt(complex(q))
    S0 = special.jv(0, z)
    S1 = 1.0 if z == 0 else 2.0 * special.jv(1, z) / z
    d0 = S0 * g0
    if p.zassenhaus:
        d0 = d0 * np.exp(q / 8.0)
    dp1 = 1j * (dZ * p.chih / (2.0 * c)) * S1 * g0
    dm1 = 1j * (dZ * p.chihbar / (2.0 * c)) * S1 * g0
    return complex(d0), complex(dp1), complex(dm1)


def wavenumbers(Nx: int, dx: float) -> np.ndarray:
    """K_m = 2 pi m / (Nx dx) for the DFT bin order m = 0..Nx/2-1, -Nx/2..-1,
    in extended precision."""
    m = np.fft.fftfreq(Nx, 1.0 / Nx).astype(np.longdouble)  # exact integers
    return TWO_PI_X * m / (np.longdouble(Nx) * np.longdouble(dx))


def propagator(p: Problem, delta: float, band: int, frac: float = 1.0):
    """Free-propagation multiplier of one band for a sub-step frac*dz:
    exp(i frac dz sqrt(k^2 - (K + band h/2)^2)), band = +1 for psi~_+ and
    -1 for psi~_-; principal root (decay) where the wave is evanescent.  The
    phase is formed and reduced modulo 2 pi in extended precision."""
    k0, h = beam_constants(p)
    k = np.longdouble(k0 * (1.0 + delta))
    K = wavenumbers(p.Nx, p.dx)
    kp = K + np.longdouble(band) * np.longdouble(h) / 2
    kz2 = k * k - kp * kp
    L = np.longdouble(frac) * np.longdouble(p.dz)
    prop = kz2 >= 0
    phi = np.where(prop, L * np.sqrt(np.where(prop, kz2, 0)), 0)
    phi = np.fmod(phi, TWO_PI_X).astype(np.float64)
    decay = np.where(prop, 0, L * np.sqrt(np.where(prop, 0, -kz2)))
    return np.exp(1j * phi - decay.astype(np.float64))


def crystal_mask(p: Problem, n: int = 0) -> np.ndarray:
    """Pi_j of step n: the general mask row p.mask[n] when one is given,
    otherwise the slab x_front <= x_j < x_front + thickness, x_j = (j - Nx/2) dx
    (the same for every step)."""
    if p.mask is not None:
        return p.mask[n]
    x = (np.arange(p.Nx) - p.Nx // 2) * p.dx
    return (x >= p.x_front) & (x < p.x_front + p.thickness)


def deformation_factor(p: Problem, u_row) -> np.ndarray:
    """exp(i h u) of Eq. Authier for one z row (u in metres along h)."""
    _, h = beam_constants(p)
    return np.exp(1j * (h * np.asarray(u_row, dtype=np.float64)))


def split_coefficients(order: int):
    """(a_i, b_i) of Eq. split-op: first order (1, 1); second order
    a = (0, 1), b = (1/2, 1/2); fourth order with t = 1/(2 - 2^(1/3))
    (printed rounded as 1.3512)."""
    if order == 1:
        return [1.0], [1.0]
    if order == 2:
        return [0.0, 1.0], [0.5, 0.5]
    if order == 4:
        t = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
        return [0.0, t, 1.0 - 2.0 * t, t], [t / 2, (1 - t) / 2, (1 - t) / 2, t / 2]
    raise ValueError("split order must be 1, 2 or 4")


def march(p: Problem, E0_in, u=None, n_steps=None, Eh_in=None,
          return_history=False):
    """Run the z-march for every slice.

    E0_in: (Nomega, Nx) complex, psi~_+ at z = 0.  Eh_in: optional psi~_- at
    z = 0 (zero by default).  u: optional (Nz, Nx) float64 displacement, row n
    used by step n.  Returns (E0_out, Eh_out), each (Nomega, Nx) complex128;
    with return_history also the list of per-step (a, b) intensities summed
    over x (for flux checks).
    """
    Nw, Nx = p.Nomega, p.Nx
    a = np.array(E0_in, dtype=np.complex128).reshape(Nw, Nx)
    b = (np.zeros_like(a) if Eh_in is None
         else np.array(Eh_in, dtype=np.complex128).reshape(Nw, Nx))
    n_steps = p.Nz if n_steps is None else int(n_steps)
    A, Bc = split_coefficients(p.split_order)

    # Per-slice, per-substep constants.
    props = []
    for ai in A:
        if ai == 0.0:
            props.append(None)
        else:
            props.append((np.stack([propagator(p, d, +1, ai) for d in p.delta]),
                          np.stack([propagator(p, d, -1, ai) for d in p.delta])))
    coup = []
    for bi in Bc:
        cc = np.array([coupling_constants(p, d, bi) for d in p.delta])
        coup.append((cc[:, 0:1], cc[:, 1:2], cc[:, 2:3]))

    hist = []
    for n in range(n_steps):
        e = None if u is None else deformation_factor(p, u[n])[None, :]
        mask = crystal_mask(p, n)[None, :]
        for i in range(len(A)):
            if props[i] is not None:
                Pp, Pm = props[i]
                a = np.fft.ifft(Pp * np.fft.fft(a, axis=-1), axis=-1)
                b = np.fft.ifft(Pm * np.fft.fft(b, axis=-1), axis=-1)
            d0, dp1, dm1 = coup[i]
            if e is None:
                a_new = d0 * a + dp1 * b
                b_new = d0 * b + dm1 * a
            else:
                a_new = d0 * a + dp1 * e * b
                b_new = d0 * b + dm1 * np.conj(e) * a
            a = np.where(mask, a_new, a)
            b = np.where(mask, b_new, b)
        if return_history:
            hist.append((np.sum(np.abs(a) ** 2, axis=-1),
                         np.sum(np.abs(b) ** 2, axis=-1)))
    if return_history:
        return a, b, hist
    return a, b
