"""Error metrics between two sets of output fields (no method arithmetic)."""

from __future__ import annotations

import numpy as np


def rel_l2(test, ref) -> float:
    """||test - ref||_2 / ||ref||_2 over all entries (complex)."""
    test = np.asarray(test, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    den = np.linalg.norm(ref)
    if den == 0.0:
        return float(np.linalg.norm(test))
    return float(np.linalg.norm(test - ref) / den)


def phase_error(test, ref, floor: float = 1e-6) -> float:
    """Intensity-weighted rms of arg(test * conj(ref)) over the cells whose
    reference intensity is at least floor * max (radians)."""
    test = np.asarray(test, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    I = np.abs(ref) ** 2
    if I.size == 0 or I.max() == 0.0:
        return 0.0
    sel = I >= floor * I.max()
    ang = np.angle(test[sel] * np.conj(ref[sel]))
    w = I[sel]
    return float(np.sqrt(np.sum(w * ang * ang) / np.sum(w)))


def per_slice_rel_l2(test, ref) -> np.ndarray:
    """relL2 of each slice (rows of a (Nomega, Nx) array)."""
    test = np.asarray(test, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    num = np.linalg.norm(test - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), num)


def report(E0_t, Eh_t, E0_r, Eh_r) -> dict:
    """relL2 over the concatenation of both fields, per field, worst slice,
    and the intensity-weighted phase error."""
    t = np.concatenate([np.ravel(E0_t), np.ravel(Eh_t)])
    r = np.concatenate([np.ravel(E0_r), np.ravel(Eh_r)])
    ps0 = per_slice_rel_l2(np.atleast_2d(E0_t), np.atleast_2d(E0_r))
    psh = per_slice_rel_l2(np.atleast_2d(Eh_t), np.atleast_2d(Eh_r))
    return dict(rel_l2=rel_l2(t, r), rel_l2_E0=rel_l2(E0_t, E0_r),
                rel_l2_Eh=rel_l2(Eh_t, Eh_r),
                worst_slice_rel_l2=float(max(ps0.max(), psh.max())),
                phase_err_rad=phase_error(t, r))
