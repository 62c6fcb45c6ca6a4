"""Plain CPU oracle of the two-beam FFT BPM z-march on a 3D grid (FP64).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product library never does.

The 3D problem has two transverse axes, x (along the reciprocal vector h,
the axis of the two angular bands) and y, and marches along z.  Section 2.1
states the step for both transverse wavenumbers (Eq. fov4 with k_x and k_y)
and says the generalisation of the two-band method to 3D is direct; the
finite-element example of Section 3.4 runs on such a grid.  Step by step, in
the paper's order, for every frequency slice:

  * Eq. fov4  -- 2D FFT over (y, x), multiply by the free-propagation phase
    exp(i dz sqrt(k^2 - k_x^2 - k_y^2)) of each band, inverse 2D FFT;
  * Eqs. fov6, fov7, fov10 -- the band envelopes psi~_+ and psi~_- carry
    +-h/2 along x, so band +-1 propagates with
    sqrt(k^2 - (K_x +- h/2)^2 - K_y^2);
  * Eq. fov10, Eqs. fov11, fov12, Eq. Authier, the Zassenhaus-like factor --
    the same pointwise 2 x 2 coupling as the 2D march (coupling constants
    from oracle.bpm), at every (x, y), with the deformation phase
    exp(+-i h u(x, y, z)) and the crystal mask.

Readings (listed with their reasons in the design notes): the crystal is the
symmetric-Bragg slab x_front <= x < x_front + thickness for every y, or a
general mask Pi(x, y, z) with one (y, x) row per step;
cos(alpha) = sqrt(1 - (h/2k)^2) as in 2D (the mean angular spectrum has no
k_y component); y_i = (i - Ny/2) dy like x; periodic window in both axes;
the splitting schemes of Eq. split-op (first, second and fourth order) with
the sub-steps of a step using that step's deformation and crystal, as in
oracle.bpm.  The propagator phase is formed and reduced modulo 2 pi in
extended precision, as in oracle.bpm.
"""

from __future__ import annotations

import math

import numpy as np

from . import bpm

__all__ = ["Problem3D", "wavenumbers_y", "propagator3d", "crystal_mask3d",
           "march3d"]


class Problem3D:
    """Parameters of one 3D problem (all slices share them except delta)."""

    def __init__(self, Nx, Ny, dx, dy, dz, Nz, chi0, chih, chihbar, theta_B,
                 lam, delta, x_front=0.0, thickness=math.inf, zassenhaus=True,
                 split_order=1, mask=None):
        self.Nx, self.Ny = int(Nx), int(Ny)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.Nz = int(Nz)
        self.chi0, self.chih, self.chihbar = complex(chi0), complex(chih), complex(chihbar)
        self.theta_B, self.lam = float(theta_B), float(lam)
        self.delta = np.atleast_1d(np.asarray(delta, dtype=np.float64))
        self.x_front, self.thickness = float(x_front), float(thickness)
        self.zassenhaus = bool(zassenhaus)
        self.split_order = int(split_order)
        # general crystal mask Pi(x, y, z): (Nz, Ny, Nx) booleans, row n used
        # by every sub-step of step n; None selects the slab
        self.mask = None if mask is None else np.asarray(mask, dtype=bool).reshape(
            self.Nz, self.Ny, self.Nx)

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(Nx=w.Nx, Ny=w.Ny, dx=w.dx, dy=w.dy, dz=w.dz, Nz=w.Nz,
                  chi0=w.chi0, chih=w.chih, chihbar=w.chihbar,
                  theta_B=w.theta_B, lam=w.lam, delta=w.delta,
                  x_front=w.x_front, thickness=w.thickness)
        kw.update(over)
        return cls(**kw)

    @property
    def Nomega(self):
        return len(self.delta)

    def along_x(self) -> bpm.Problem:
        """The 2D problem with the same x grid and physics (its coupling
        constants, beam constants and wavenumbers are those of this one)."""
        return bpm.Problem(self.Nx, self.dx, self.dz, self.Nz, self.chi0,
                           self.chih, self.chihbar, self.theta_B, self.lam,
                           self.delta, self.x_front, self.thickness,
                           self.zassenhaus, split_order=self.split_order)


def wavenumbers_y(Ny: int, dy: float) -> np.ndarray:
    """K_y = 2 pi m / (Ny dy) in DFT bin order, extended precision."""
    m = np.fft.fftfreq(Ny, 1.0 / Ny).astype(np.longdouble)
    return bpm.TWO_PI_X * m / (np.longdouble(Ny) * np.longdouble(dy))


def propagator3d(p: Problem3D, delta: float, band: int, frac: float = 1.0) -> np.ndarray:
    """(Ny, Nx) free-propagation multiplier of one band for a sub-step of
    frac*dz: exp(i frac dz sqrt(k^2 - (K_x + band h/2)^2 - K_y^2)),
    principal root (decay) where evanescent; the phase reduced modulo 2 pi
    in extended precision."""
    k0, h = bpm.beam_constants(p.along_x())
    k = np.longdouble(k0 * (1.0 + delta))
    Kx = bpm.wavenumbers(p.Nx, p.dx)[None, :]
    Ky = wavenumbers_y(p.Ny, p.dy)[:, None]
    kp = Kx + np.longdouble(band) * np.longdouble(h) / 2
    kz2 = k * k - kp * kp - Ky * Ky
    L = np.longdouble(frac) * np.longdouble(p.dz)
    prop = kz2 >= 0
    phi = np.where(prop, L * np.sqrt(np.where(prop, kz2, 0)), 0)
    phi = np.fmod(phi, bpm.TWO_PI_X).astype(np.float64)
    decay = np.where(prop, 0, L * np.sqrt(np.where(prop, 0, -kz2)))
    return np.exp(1j * phi - decay.astype(np.float64))


def crystal_mask3d(p: Problem3D, n: int = 0) -> np.ndarray:
    """(Ny, Nx) crystal mask of step n: the general mask p.mask[n] when one
    is given, otherwise the slab x_front <= x_j < x_front + thickness,
    x_j = (j - Nx/2) dx, the same for every y and step."""
    if p.mask is not None:
        return p.mask[n]
    x = (np.arange(p.Nx) - p.Nx // 2) * p.dx
    row = (x >= p.x_front) & (x < p.x_front + p.thickness)
    return np.broadcast_to(row, (p.Ny, p.Nx))


def march3d(p: Problem3D, E0_in, u=None, n_steps=None, Eh_in=None):
    """Run the 3D z-march for every slice.

    E0_in: (Nomega, Ny, Nx) complex, psi~_+ at z = 0; Eh_in: optional psi~_-
    at z = 0 (zero by default).  u: optional (Nz, Ny, Nx) float64
    displacement along h, [n] used by step n.  Returns (E0_out, Eh_out), each
    (Nomega, Ny, Nx) complex128."""
    Nw, Ny, Nx = p.Nomega, p.Ny, p.Nx
    a = np.array(E0_in, dtype=np.complex128).reshape(Nw, Ny, Nx)
    b = (np.zeros_like(a) if Eh_in is None
         else np.array(Eh_in, dtype=np.complex128).reshape(Nw, Ny, Nx))
    n_steps = p.Nz if n_steps is None else int(n_steps)
    p2 = p.along_x()
    _, h = bpm.beam_constants(p2)
    A, Bc = bpm.split_coefficients(p.split_order)
    props = [None if ai == 0.0 else
             (np.stack([propagator3d(p, d, +1, ai) for d in p.delta]),
              np.stack([propagator3d(p, d, -1, ai) for d in p.delta]))
             for ai in A]
    coup = []
    for bi in Bc:
        cc = np.array([bpm.coupling_constants(p2, d, bi) for d in p.delta])
        coup.append(tuple(cc[:, i][:, None, None] for i in range(3)))
    for n in range(n_steps):
        e = None if u is None else np.exp(1j * (h * np.asarray(u[n], dtype=np.float64)))[None]
        mask = crystal_mask3d(p, n)[None]
        for i in range(len(A)):
            if props[i] is not None:
                Pp, Pm = props[i]
                a = np.fft.ifft2(Pp * np.fft.fft2(a, axes=(-2, -1)), axes=(-2, -1))
                b = np.fft.ifft2(Pm * np.fft.fft2(b, axes=(-2, -1)), axes=(-2, -1))
            d0, dp1, dm1 = coup[i]
            if e is None:
                a_new = d0 * a + dp1 * b
                b_new = d0 * b + dm1 * a
            else:
                a_new = d0 * a + dp1 * e * b
                b_new = d0 * b + dm1 * np.conj(e) * a
            a = np.where(mask, a_new, a)
            b = np.where(mask, b_new, b)
    return a, b
