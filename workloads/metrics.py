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


def max_err(test, ref) -> float:
    """max |test - ref| / max |ref| over all entries (elementwise error
    against the field's scale; the absolute error if ref is zero)."""
    test = np.asarray(test, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    if test.size == 0:
        return 0.0
    num = float(np.max(np.abs(test - ref)))
    den = float(np.max(np.abs(ref)))
    return num / den if den > 0.0 else num


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
    """Errors of the outputs (E0_t, Eh_t) against (E0_r, Eh_r):
      rel_l2              over the concatenation of both fields, all slices;
      rel_l2_E0, _Eh      each field on its own, all slices;
      worst_slice_rel_l2  the worst slice's result (both fields of it);
      worst_slice_field_rel_l2  the worst single (slice, field) row, measured
                          against that row's own norm;
      max_err             max elementwise |error| / max |ref| over both fields;
      max_err_E0, _Eh     the same per field, each against its own maximum;
      phase_err_rad       intensity-weighted rms phase error."""
    a_t, b_t = np.atleast_2d(E0_t), np.atleast_2d(Eh_t)
    a_r, b_r = np.atleast_2d(E0_r), np.atleast_2d(Eh_r)
    t = np.concatenate([a_t.ravel(), b_t.ravel()])
    r = np.concatenate([a_r.ravel(), b_r.ravel()])
    ps0 = per_slice_rel_l2(a_t, a_r)
    psh = per_slice_rel_l2(b_t, b_r)
    both = per_slice_rel_l2(np.concatenate([a_t, b_t], axis=-1),
                            np.concatenate([a_r, b_r], axis=-1))
    return dict(rel_l2=rel_l2(t, r), rel_l2_E0=rel_l2(a_t, a_r),
                rel_l2_Eh=rel_l2(b_t, b_r),
                worst_slice_rel_l2=float(both.max()),
                worst_slice_field_rel_l2=float(max(ps0.max(), psh.max())),
                max_err=max_err(t, r), max_err_E0=max_err(a_t, a_r),
                max_err_Eh=max_err(b_t, b_r),
                phase_err_rad=phase_error(t, r))


PARITY_KEYS = ("rel_l2", "rel_l2_E0", "rel_l2_Eh", "max_err", "max_err_E0",
               "max_err_Eh")


def within(r: dict, tol: float, phase_tol: float | None = None,
           keys=PARITY_KEYS) -> list:
    """Names of the metrics of a report that exceed tol (and the phase error
    that exceeds phase_tol, if given); empty when all are within."""
    bad = [k for k in keys if not r[k] <= tol]
    if phase_tol is not None and not r["phase_err_rad"] <= phase_tol:
        bad.append("phase_err_rad")
    return bad
