"""Pins of the oracle's general crystal mask Pi(x, z): a mask equal to the
slab reproduces the slab march exactly, an empty mask is free propagation,
and a crystal block in z (Laue geometry, the whole window filled for a range
of steps) gives the textbook Pendelloesung of a plane wave at the Bragg
condition, |psi_h|^2 = sin^2(pi D / Lambda), Lambda = lambda cos(theta_B) /
|chi_h| (symmetric Laue case, no absorption)."""

import math

import numpy as np

import oracle as O
import workloads as W


def _problem(w, **kw):
    return O.Problem.from_workload(w, **kw)


def test_slab_shaped_mask_equals_slab():
    w = W.small(Nx=256, Nz=30, Nomega=2, seed=11, x_front=-20e-6, thickness=40e-6)
    x = (np.arange(w.Nx) - w.Nx // 2) * w.dx
    slab = (x >= w.x_front) & (x < w.x_front + w.thickness)
    m = np.broadcast_to(slab, (w.Nz, w.Nx))
    a1, b1 = O.march(_problem(w), w.E0_in, w.u)
    a2, b2 = O.march(_problem(w, mask=m), w.E0_in, w.u)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_empty_mask_is_free_propagation():
    w = W.small(Nx=256, Nz=20, Nomega=2, seed=12)
    a1, b1 = O.march(_problem(w, x_front=1.0, thickness=1.0), w.E0_in, w.u)
    a2, b2 = O.march(_problem(w, mask=np.zeros((w.Nz, w.Nx), bool)), w.E0_in, w.u)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    assert np.all(b2 == 0)


def test_laue_block_pendelloesung():
    lam, th = 1.24e-10, math.pi / 4
    chih = 3.8e-6
    Lam = lam * math.cos(th) / chih          # Pendelloesung distance (period of |psi_h|^2)
    Nx, dz = 64, 0.02e-6
    n1 = 50
    for D_over in (0.13, 0.25, 0.41, 0.5, 0.77):
        n_cr = int(round(D_over * Lam / dz))
        Nz = n1 + n_cr + 20
        m = np.zeros((Nz, Nx), bool)
        m[n1:n1 + n_cr] = True
        p = O.Problem(Nx, 0.5e-6, dz, Nz, 0.0, chih, chih, th, lam, [0.0], mask=m)
        a, b = O.march(p, np.ones((1, Nx), complex))
        D = n_cr * dz
        Ih = np.mean(np.abs(b) ** 2)
        assert abs(Ih - math.sin(math.pi * D / Lam) ** 2) < 2e-4, (D_over, Ih)
        assert abs(np.mean(np.abs(a) ** 2) + Ih - 1) < 1e-6     # no absorption
