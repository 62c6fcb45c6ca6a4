"""Pins of the oracle's time <-> frequency pair (Eq. tdp, Section 3): exact
identities of the discrete Fourier pair, the analytic transform of a
Gaussian, the vacuum group delay of a marched pulse, and the wake of a pulse
reflected by a thick perfect crystal, whose displacement along the reflected
beam's cross-section grows at c cot(theta_B) (the slope the paper draws on
its spatio-temporal map)."""

import math

import numpy as np
import pytest

import oracle as O
from oracle import pulse as P
import workloads.configs as W
from pulse_analysis import wake_slope

C = P.C_LIGHT


def test_round_trip_is_identity_and_parseval_holds():
    rng = np.random.default_rng(3)
    f = rng.normal(size=(64, 5)) + 1j * rng.normal(size=(64, 5))
    dt = 0.7e-15
    g = P.to_frequency(f, dt)
    assert np.max(np.abs(P.to_time(g, dt) - f)) < 1e-13 * np.max(np.abs(f))
    # dt sum |f|^2 = (dOmega / 2 pi) sum |g|^2
    dOm = 2 * np.pi / (64 * dt)
    lhs = dt * np.sum(np.abs(f) ** 2, axis=0)
    rhs = dOm / (2 * np.pi) * np.sum(np.abs(g) ** 2, axis=0)
    assert np.allclose(lhs, rhs, rtol=1e-13)


def test_single_sample_and_pure_tone_transform_exactly():
    N, dt = 32, 1e-15
    t = P.time_grid(N, dt)
    W_ = P.frequency_grid(N, dt)
    # a sample at t_i transforms to dt exp(+i Omega t_i) (the printed sign)
    f = np.zeros((N, 1), complex)
    f[5, 0] = 1.0
    assert np.allclose(P.to_frequency(f, dt)[:, 0], dt * np.exp(1j * W_ * t[5]),
                       rtol=0, atol=1e-28)
    # exp(-i Omega_j t) transforms to N dt at slice j only
    g = P.to_frequency(np.exp(-1j * W_[9] * t)[:, None], dt)[:, 0]
    expect = np.zeros(N, complex)
    expect[9] = N * dt
    assert np.max(np.abs(g - expect)) < 1e-12 * N * dt


def test_gaussian_transforms_to_gaussian_with_shift_phase():
    """FT of exp(-(t-t0)^2/2s^2) with exp(+i Omega t) is
    s sqrt(2 pi) exp(-Omega^2 s^2 / 2) exp(+i Omega t0)."""
    N, dt, s, t0 = 256, 1e-15, 8e-15, 12e-15
    t = P.time_grid(N, dt)
    Om = P.frequency_grid(N, dt)
    g = P.to_frequency(np.exp(-0.5 * ((t - t0) / s) ** 2)[:, None], dt)[:, 0]
    exact = s * math.sqrt(2 * math.pi) * np.exp(-0.5 * (Om * s) ** 2) * np.exp(1j * Om * t0)
    assert np.max(np.abs(g - exact)) < 1e-12 * np.max(np.abs(exact))


def test_detuning_grid_is_frequency_offset_over_carrier():
    N, dt, lam = 16, 2e-15, 1.24e-10
    om0 = 2 * np.pi * C / lam
    assert np.allclose(P.detuning(N, dt, lam) * om0, P.frequency_grid(N, dt), rtol=1e-15)
    assert P.frequency_grid(N, dt)[N // 2] == 0.0


def _march_pulse(Nx, Nz, N, dt, sig, w0, x0, theta, x_front=0.0, thickness=math.inf):
    dx = dz = 0.5e-6
    lam = W.LAMBDA
    f = W.pulse_field(Nx, dx, N, dt, lam, theta, theta, sig, x0=x0, w0=w0)
    prob = O.Problem(Nx, dx, dz, Nz, W.CHI0, W.CHIH, W.CHIH, theta, lam,
                     P.detuning(N, dt, lam), x_front=x_front, thickness=thickness)
    a, b = O.march(prob, P.to_frequency(f, dt))
    return P.to_time(a, dt), P.to_time(b, dt)


def test_vacuum_pulse_arrives_after_group_delay_at_walked_off_position():
    """In vacuum the pulse moves along (sin theta, cos theta) at c: at z = L
    its centre is at x0 + L tan(theta) and arrives at L / (c cos(theta))
    (d kz / d omega = 1 / (c cos alpha) at the carrier)."""
    Nx, Nz, N, dt, sig, theta = 512, 20, 256, 1e-15, 6e-15, W.THETA_B
    x0, w0 = -30e-6, 15e-6
    a, _ = _march_pulse(Nx, Nz, N, dt, sig, w0, x0, theta, x_front=1.0, thickness=1.0)
    L = Nz * 0.5e-6
    x = W.x_grid(Nx, 0.5e-6)
    I = np.abs(a) ** 2
    xc = np.sum(I * x[None, :]) / np.sum(I)
    assert abs(xc - (x0 + L * math.tan(theta))) < 0.01e-6
    t = P.time_grid(N, dt)
    row = np.abs(a[:, np.argmin(np.abs(x - xc))]) ** 2
    # circular centroid of the arrival time at the beam centre
    T = N * dt
    ph = np.angle(np.sum(row * np.exp(2j * np.pi * t / T)))
    t_arr = ph * T / (2 * np.pi)
    expect = L / (C * math.cos(theta))      # path L / cos(theta) at c
    expect = (expect + T / 2) % T - T / 2
    assert abs(t_arr - expect) < 0.05e-15


def _wake_slope(theta_deg, Nz):
    theta = math.radians(theta_deg)
    Nx, N, dt, sig = 1024, 512, 1e-15, 2e-15
    _, b = _march_pulse(Nx, Nz, N, dt, sig, 20e-6, -40e-6, theta)
    return wake_slope(b, W.x_grid(Nx, 0.5e-6), P.time_grid(N, dt), theta)


@pytest.mark.slow
@pytest.mark.parametrize("theta_deg,Nz", [(45.0, 300), (30.0, 600)])
def test_reflected_wake_moves_at_c_cot_theta(theta_deg, Nz):
    slope = _wake_slope(theta_deg, Nz)
    expect = C / math.tan(math.radians(theta_deg))
    assert abs(slope / expect - 1) < 0.03, (slope, expect)
