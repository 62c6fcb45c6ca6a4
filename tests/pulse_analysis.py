"""Analysis of spatio-temporal maps of a reflected pulse (test helper; no
propagation arithmetic)."""

import math

import numpy as np

C = 299792458.0


def wake_slope(b_t, x, t, theta, half_width=140e-6, fit=(12e-15, 124e-15)):
    """Rate at which the reflected field's wake moves along the reflected
    beam's cross-section.  Beam-frame delay tau = t - t0 + (x - xc)
    sin(theta)/c and cross-section coordinate x_perp = (x - xc) cos(theta)
    (unit vector (cos theta, sin theta), towards the crystal side), with
    (t0, xc) the intensity peak; the intensity centroid of x_perp in 4 fs
    bins of tau is fitted linearly over `fit`."""
    I = np.abs(b_t) ** 2
    T = len(t) * (t[1] - t[0])
    it0, ix0 = np.unravel_index(I.argmax(), I.shape)
    sel = np.abs(x - x[ix0]) < half_width
    xs, Is = x[sel], I[:, sel]
    tau = (t[:, None] - t[it0]) + (xs[None, :] - x[ix0]) * math.sin(theta) / C
    tau = np.mod(tau + T / 4, T) - T / 4
    xp = np.broadcast_to(((xs - x[ix0]) * math.cos(theta))[None, :], Is.shape)
    edges = np.arange(fit[0], fit[1], 4e-15)
    k = np.digitize(tau.ravel(), edges)
    taus, cents = [], []
    for j in range(1, len(edges)):
        m = k == j
        p = Is.ravel()[m].sum()
        taus.append(edges[j - 1])
        cents.append((Is.ravel()[m] * xp.ravel()[m]).sum() / p)
    return np.polyfit(taus, cents, 1)[0]
