"""Pins of the 3D oracle (oracle/bpm3d.py) against quantities fixed
independently of its code: the pinned 2D oracle it must reduce to exactly,
a brute-force 2D DFT on a non-power-of-two grid, the analytic 3D Gaussian
beam in free space, and the closed-form mode coupling of a uniform strain
along y.  A plausible slip (a transposed (y, x) axis, a dropped K_y term, a
wrong 1/cos factor in y, a wrong fftfreq order for odd sizes) fails at least
one of them."""

import math

import numpy as np
import pytest

import oracle as O
from closed_forms import dft_brute, gaussian_beam_3d

LAM = 1.24e-10
TH = math.pi / 4
CHI0 = complex(-1.5e-5, 1e-8)
CHIH = complex(3.8e-6, 0.9e-8)
VACUUM = dict(x_front=1.0, thickness=1.0)
FILLED = dict(x_front=-1.0, thickness=math.inf)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def rand_field(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def grid(N, d):
    return (np.arange(N) - N // 2) * d


def p3(Nx, Ny, Nz, delta=(0.0,), dx=0.5e-6, dy=0.5e-6, dz=0.5e-6, chih=CHIH,
       chihbar=CHIH, **kw):
    return O.Problem3D(Nx, Ny, dx, dy, dz, Nz, CHI0, chih, chihbar, TH, LAM,
                       list(delta), **kw)


@pytest.mark.parametrize("Nx", [64, 90])
def test_one_row_is_the_2d_march(Nx):
    """Ny = 1: the 3D march is the pinned 2D march (K_y = 0 only), with a
    partial slab, deformation and two slices."""
    rng = np.random.default_rng(Nx)
    Nz, deltas = 17, [0.0, 4e-6]
    p = p3(Nx, 1, Nz, deltas, x_front=-5e-6, thickness=12e-6)
    E0 = rand_field(rng, 2, 1, Nx)
    u = rng.normal(scale=3e-11, size=(Nz, 1, Nx))
    a, b = O.march3d(p, E0, u)
    q = O.Problem(Nx, 0.5e-6, 0.5e-6, Nz, CHI0, CHIH, CHIH, TH, LAM, deltas,
                  x_front=-5e-6, thickness=12e-6)
    a2, b2 = O.march(q, E0[:, 0, :], u[:, 0, :])
    assert rel(a[:, 0], a2) < 1e-14 and rel(b[:, 0], b2) < 1e-13


@pytest.mark.parametrize("order", [2, 4])
def test_one_row_is_the_2d_march_every_order(order):
    """Ny = 1 with the second- and fourth-order schemes of Eq. split-op is the
    pinned 2D march with the same scheme (sub-step propagators, sub-step
    coupling constants, the step's deformation and slab for every
    sub-step)."""
    rng = np.random.default_rng(order)
    Nx, Nz, deltas = 72, 11, [0.0, -3e-6]
    p = p3(Nx, 1, Nz, deltas, x_front=-6e-6, thickness=14e-6, split_order=order)
    E0 = rand_field(rng, 2, 1, Nx)
    u = rng.normal(scale=3e-11, size=(Nz, 1, Nx))
    a, b = O.march3d(p, E0, u)
    q = O.Problem(Nx, 0.5e-6, 0.5e-6, Nz, CHI0, CHIH, CHIH, TH, LAM, deltas,
                  x_front=-6e-6, thickness=14e-6, split_order=order)
    a2, b2 = O.march(q, E0[:, 0, :], u[:, 0, :])
    assert rel(a[:, 0], a2) < 1e-13 and rel(b[:, 0], b2) < 1e-13


def _conv_errors_3d(order, factors=(1, 2, 4)):
    """Relative error of the 3D march over a fixed depth against a run with
    32 times smaller steps: a beam that is Gaussian in both x and y, at the
    Bragg angle, in an unbounded crystal."""
    Nx, Ny, dx, dy, Z = 128, 16, 0.5e-6, 0.5e-6, 40e-6
    x, y = grid(Nx, dx), grid(Ny, dy)
    k0 = 2 * math.pi / LAM
    h = 2 * k0 * math.sin(TH)
    E0 = (np.exp(-(y / 2e-6) ** 2)[:, None]
          * (np.exp(-((x + 10e-6) / 8e-6) ** 2)
             * np.exp(1j * (k0 * math.sin(TH + 1.5e-5) - h / 2) * x))[None, :])[None]

    def run(dz):
        p = O.Problem3D(Nx, Ny, dx, dy, dz, int(round(Z / dz)), CHI0, CHIH, CHIH, TH,
                        LAM, [0.0], split_order=order, **FILLED)
        a, b = O.march3d(p, E0)
        return np.concatenate([a.ravel(), b.ravel()])

    ref = run(0.5e-6 / 32)
    return [rel(run(0.5e-6 / f), ref) for f in factors]


@pytest.mark.parametrize("order,lo,hi", [(1, 0.9, 1.25), (2, 1.8, 2.2)])
def test_convergence_order_3d(order, lo, hi):
    """The scheme's order survives the y axis: first order for Lie splitting
    (measured slopes 1.12, 1.12), second for Strang (2.01, 2.02)."""
    e = _conv_errors_3d(order)
    for i in range(len(e) - 1):
        assert lo < math.log2(e[i] / e[i + 1]) < hi, e


def test_fourth_order_3d_beats_second_order():
    """The fourth-order product converges at least at second order (its B
    step, the three-term Jacobi-Anger expansion, is accurate to second order,
    so the asymptotic slope is 2, as in 2D; measured 3.31 then 1.73 while the
    coarse steps are still dominated by the A-B splitting error), and its
    error stays below Strang's at every step size."""
    e4, e2 = _conv_errors_3d(4), _conv_errors_3d(2)
    for i in range(len(e4) - 1):
        assert 1.6 < math.log2(e4[i] / e4[i + 1]) < 3.6, e4
    assert all(a < 0.3 * b for a, b in zip(e4, e2)), (e4, e2)


def test_mask_shaped_like_the_slab_is_the_slab():
    """A general mask that reproduces the slab in every step gives the slab
    march bitwise; an empty mask is free propagation."""
    rng = np.random.default_rng(21)
    Nx, Ny, Nz = 40, 4, 9
    kw = dict(x_front=-4e-6, thickness=9e-6)
    p = p3(Nx, Ny, Nz, [0.0, 2e-6], **kw)
    E0 = rand_field(rng, 2, Ny, Nx)
    u = rng.normal(scale=3e-11, size=(Nz, Ny, Nx))
    slab = np.broadcast_to(O.crystal_mask3d(p), (Nz, Ny, Nx))
    a, b = O.march3d(p, E0, u)
    am, bm = O.march3d(p3(Nx, Ny, Nz, [0.0, 2e-6], mask=slab, **kw), E0, u)
    assert np.array_equal(a, am) and np.array_equal(b, bm)
    av, bv = O.march3d(p3(Nx, Ny, Nz, [0.0, 2e-6], **VACUUM), E0, u)
    ae, be = O.march3d(p3(Nx, Ny, Nz, [0.0, 2e-6], mask=np.zeros((Nz, Ny, Nx)), **kw), E0, u)
    assert np.array_equal(av, ae) and np.array_equal(bv, be)


def test_one_row_with_a_mask_is_the_masked_2d_march():
    """Ny = 1 with a general mask that changes from step to step is the
    pinned masked 2D march (Laue block, shaped entrance)."""
    rng = np.random.default_rng(22)
    Nx, Nz = 64, 15
    m2 = rng.random((Nz, Nx)) < 0.6
    E0 = rand_field(rng, 1, 1, Nx)
    u = rng.normal(scale=3e-11, size=(Nz, 1, Nx))
    a, b = O.march3d(p3(Nx, 1, Nz, mask=m2[:, None, :], split_order=2), E0, u)
    q = O.Problem(Nx, 0.5e-6, 0.5e-6, Nz, CHI0, CHIH, CHIH, TH, LAM, [0.0],
                  split_order=2, mask=m2)
    a2, b2 = O.march(q, E0[:, 0, :], u[:, 0, :])
    assert rel(a[:, 0], a2) < 1e-13 and rel(b[:, 0], b2) < 1e-13


@pytest.mark.parametrize("Ny", [6, 5])
def test_y_independent_problem_has_2d_rows(Ny):
    """A field and a displacement that do not depend on y stay independent
    of y, and every row is the 2D march (even and odd Ny)."""
    rng = np.random.default_rng(Ny)
    Nx, Nz = 48, 13
    row = rand_field(rng, 1, Nx)
    urow = rng.normal(scale=3e-11, size=(Nz, Nx))
    p = p3(Nx, Ny, Nz, x_front=-3e-6, thickness=math.inf)
    a, b = O.march3d(p, np.repeat(row[:, None, :], Ny, axis=1),
                     np.repeat(urow[:, None, :], Ny, axis=1))
    q = O.Problem(Nx, 0.5e-6, 0.5e-6, Nz, CHI0, CHIH, CHIH, TH, LAM, [0.0],
                  x_front=-3e-6, thickness=math.inf)
    a2, b2 = O.march(q, row, urow)
    for i in range(Ny):
        assert rel(a[0, i], a2[0]) < 1e-13 and rel(b[0, i], b2[0]) < 1e-13


@pytest.mark.parametrize("Ny,Nx", [(5, 6), (4, 7)])
def test_vacuum_step_is_brute_force_2d_dft(Ny, Nx):
    """One free step on a tiny non-power-of-two grid equals the brute-force
    2D DFT, the band propagator on (K_y, K_x), and the inverse 2D DFT with
    1/(Nx Ny), for both bands."""
    rng = np.random.default_rng(3)
    p = p3(Nx, Ny, 1, [2e-6], **VACUUM)
    a0, b0 = rand_field(rng, 1, Ny, Nx), rand_field(rng, 1, Ny, Nx)
    a, b = O.march3d(p, a0, Eh_in=b0)

    def dft2(x):
        return dft_brute(dft_brute(x).T).T          # rows, then columns

    for band, x0, x1 in ((+1, a0, a), (-1, b0, b)):
        P = O.propagator3d(p, 2e-6, band)
        X = dft2(x0[0]) * P
        back = np.conj(dft2(np.conj(X))) / (Nx * Ny)
        assert rel(x1[0], back) < 1e-13


@pytest.mark.parametrize("band", [+1, -1])
def test_free_space_gaussian_3d(band):
    """Analytic 3D Gaussian beam (non-power-of-two grid in both axes): walk
    off along x with tan(theta), spreading with z / cos^3 theta along x and
    z / cos(theta) along y."""
    Nx, Ny, Nz = 480, 150, 150
    dx, dy, dz = 0.5e-6, 0.125e-6, 0.5e-6
    x, y = grid(Nx, dx), grid(Ny, dy)
    x0, y0, w0x, w0y = -40e-6 * band, 1.0e-6, 20e-6, 1.5e-6
    psi0 = (np.exp(-((y - y0) / w0y) ** 2)[:, None]
            * np.exp(-((x - x0) / w0x) ** 2)[None, :])[None]
    p = p3(Nx, Ny, Nz, dx=dx, dy=dy, dz=dz, **VACUUM)
    if band > 0:
        out, other = O.march3d(p, psi0)
    else:
        other, out = O.march3d(p, np.zeros_like(psi0), Eh_in=psi0)
    k = 2 * math.pi / LAM
    z = Nz * dz
    exact = gaussian_beam_3d(x, y, z, x0, y0, w0x, w0y, k, TH, band)
    assert rel(out[0], exact) < 2e-6
    assert np.max(abs(other)) == 0.0
    # the y spreading uses 1/cos(theta), not the 1/cos^3 of the band axis
    c = math.cos(TH)
    wrong = gaussian_beam_3d(x, y, z * c * c, x0, y0, w0x, w0y, k, TH, band)
    wrong *= exact[Ny // 2, Nx // 2] / wrong[Ny // 2, Nx // 2]
    assert rel(out[0], wrong) > 1e-4
    cen = np.sum(x[None, :] * abs(out[0]) ** 2) / np.sum(abs(out[0]) ** 2)
    assert abs(cen - (x0 + band * z)) < 1e-9


@pytest.mark.parametrize("m", [3, -2])
def test_uniform_strain_along_y_couples_shifted_y_modes(m):
    """u = g y with h g Ny dy = 2 pi m: exp(+ihu) moves psi~_- by +m bins of
    K_y into psi~_+ and exp(-ihu) the reverse, for every K_x (a u with its
    (y, x) axes swapped would shift K_x instead)."""
    rng = np.random.default_rng(11)
    Nx, Ny, Nz, dy = 10, 16, 9, 0.5e-6
    p = p3(Nx, Ny, Nz, dy=dy, **FILLED)
    h = 2 * (2 * math.pi / LAM) * math.sin(TH)
    g = 2 * math.pi * m / (h * Ny * dy)
    u = np.broadcast_to((g * grid(Ny, dy))[:, None], (Nz, Ny, Nx))
    a0, b0 = rand_field(rng, 1, Ny, Nx), rand_field(rng, 1, Ny, Nx)
    a, b = O.march3d(p, a0, u, Eh_in=b0)
    Pp, Pm = O.propagator3d(p, 0.0, +1), O.propagator3d(p, 0.0, -1)
    d0, dp1, dm1 = O.coupling_constants(p.along_x(), 0.0)
    s = np.exp(-1j * math.pi * m)      # y origin at i = Ny/2
    A0, B0 = np.fft.fft2(a0[0]), np.fft.fft2(b0[0])
    A, B = np.empty_like(A0), np.empty_like(B0)
    for ky in range(Ny):
        kb = (ky - m) % Ny
        for kx in range(Nx):
            step = np.array([[d0 * Pp[ky, kx], dp1 * s * Pm[kb, kx]],
                             [dm1 * np.conj(s) * Pp[ky, kx], d0 * Pm[kb, kx]]])
            A[ky, kx], B[kb, kx] = (np.linalg.matrix_power(step, Nz)
                                    @ np.array([A0[ky, kx], B0[kb, kx]]))
    assert rel(a[0], np.fft.ifft2(A)) < 1e-11
    assert rel(b[0], np.fft.ifft2(B)) < 1e-11


def test_vacuum_3d_is_unitary():
    rng = np.random.default_rng(2)
    p = p3(60, 12, 9, [0.0, -3e-6], **VACUUM)
    a0, b0 = rand_field(rng, 2, 12, 60), rand_field(rng, 2, 12, 60)
    a, b = O.march3d(p, a0, Eh_in=b0)
    assert abs(np.sum(abs(a) ** 2) / np.sum(abs(a0) ** 2) - 1) < 1e-13
    assert abs(np.sum(abs(b) ** 2) / np.sum(abs(b0) ** 2) - 1) < 1e-13
