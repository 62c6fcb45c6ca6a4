"""Closed forms used to pin the oracle.  Written from textbook physics and
mathematics, independently of oracle/ (which they never import)."""

from __future__ import annotations

import math

import numpy as np


def dft_brute(x):
    """Unnormalised forward DFT X_m = sum_j x_j exp(-2 pi i j m / N), O(N^2)."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[-1]
    j = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(j, j) / N)
    return x @ W.T


def gaussian_beam_2d(x, z, x0, w0, k, theta, band=+1):
    """Envelope of a 2D Gaussian beam exp(-(x-x0)^2/w0^2) after free
    propagation over z, for a band whose carrier travels at angle +-theta to z.

    Expanding kz(K) = sqrt(k^2 - (K + band*k sin(theta))^2) to second order in
    the envelope wavenumber K gives kz = k cos(theta) - band tan(theta) K -
    K^2 / (2 k cos^3 theta); the Fourier integral of the Gaussian is then
    exact: walk-off band*z*tan(theta) and Fresnel spreading with effective
    distance z / cos^3(theta).  The neglected cubic term is ~1e-11 rad for the
    sizes used in the tests."""
    c = math.cos(theta)
    A = w0 * w0 / 4.0 + 1j * z / (2.0 * k * c ** 3)
    X = x - x0 - band * z * math.tan(theta)
    return np.exp(1j * k * c * z) * (w0 / (2.0 * np.sqrt(A))) * np.exp(-X * X / (4.0 * A))


def darwin_reflectivity(dtheta, chi0, chih, chihbar, theta_B):
    """Thick-crystal symmetric-Bragg reflectivity (sigma polarisation) from
    two-beam dynamical theory: eta = (dtheta sin 2thetaB + chi0)/sqrt(chih
    chihbar), R = |chih/chihbar| |eta -+ sqrt(eta^2 - 1)|^2 with the root of
    modulus <= 1."""
    dtheta = np.asarray(dtheta, dtype=np.float64)
    s = np.sqrt(complex(chih) * complex(chihbar))
    eta = (dtheta * math.sin(2 * theta_B) + chi0) / s
    r = np.sqrt(eta * eta - 1 + 0j)
    x1 = eta + r
    x2 = eta - r
    x = np.where(np.abs(x1) <= np.abs(x2), x1, x2)
    return abs(chih / chihbar) * np.abs(x) ** 2


def fourier_coefficients(f, nmax=1, M=64):
    """c_n = (1/2pi) int f(t) e^{-int} dt for |n| <= nmax by M-point
    trapezoid (exact to rounding for band-limited periodic f)."""
    t = 2 * np.pi * np.arange(M) / M
    vals = f(t)
    return {n: complex(np.mean(vals * np.exp(-1j * n * t)))
            for n in range(-nmax, nmax + 1)}


def gaussian_beam_3d(x, y, z, x0, y0, w0x, w0y, k, theta, band=+1):
    """Envelope of exp(-(x-x0)^2/w0x^2 - (y-y0)^2/w0y^2) after free
    propagation over z on a 3D grid (rows y, columns x), band carrier along x.

    To second order in the envelope wavenumbers (K_x, K_y),
    sqrt(k^2 - (K_x + band k sin(theta))^2 - K_y^2) = k cos(theta)
    - band tan(theta) K_x - K_x^2 / (2 k cos^3 theta) - K_y^2 / (2 k cos theta),
    which separates: the x factor is the 2D beam (walk-off and Fresnel
    spreading with z / cos^3 theta), the y factor a Fresnel Gaussian with
    effective distance z / cos(theta).  The neglected terms (K_x^3 and
    K_x K_y^2) are below 1e-9 rad for the sizes used in the tests."""
    c = math.cos(theta)
    gx = gaussian_beam_2d(x, z, x0, w0x, k, theta, band)
    Ay = w0y * w0y / 4.0 + 1j * z / (2.0 * k * c)
    Y = np.asarray(y) - y0
    gy = (w0y / (2.0 * np.sqrt(Ay))) * np.exp(-Y * Y / (4.0 * Ay))
    return gy[:, None] * gx[None, :]
