"""Kernel invariants and tolerance gates used by the parity tests.

Gate A (the stated tolerance): |dK| <= 1e-5 everywhere, and |dK| <= 1e-3 K
where the reference K > 1e-8.
Gate B (log domain, needed because most off-diagonal K_q at d >= 64 are far
below 1e-8 and gate A cannot see them): |d ln K_q| <= 1e-3.
Invariants of a Gram matrix of normalised states (Eq. (7)) and of Eq. (3):
unit diagonal, symmetry, values in [0, 1], positive semidefinite.
"""
import numpy as np

ABS_TOL = 1e-5
REL_TOL = 1e-3
REL_FLOOR = 1e-8
LN_TOL = 1e-3


def gate_a(k_test, k_ref, abs_tol=ABS_TOL, rel_tol=REL_TOL, floor=REL_FLOOR):
    k_test = np.asarray(k_test, dtype=np.float64)
    k_ref = np.asarray(k_ref, dtype=np.float64)
    d = np.abs(k_test - k_ref)
    big = k_ref > floor
    rel = np.max(d[big] / k_ref[big]) if big.any() else 0.0
    ok = bool(np.all(d <= abs_tol) and rel <= rel_tol)
    return ok, float(d.max() if d.size else 0.0), float(rel)


def gate_b(ln_test, ln_ref, tol=LN_TOL):
    ln_test = np.asarray(ln_test, dtype=np.float64)
    ln_ref = np.asarray(ln_ref, dtype=np.float64)
    both_inf = np.isneginf(ln_test) & np.isneginf(ln_ref)
    with np.errstate(invalid="ignore"):
        d = np.where(both_inf, 0.0, np.abs(ln_test - ln_ref))
    d = np.where(np.isnan(d), np.inf, d)
    return bool(np.all(d <= tol)), float(d.max() if d.size else 0.0)


def invariants(K, diag_tol=1e-10, sym_tol=1e-12, psd_tol=None):
    """Check a square Gram matrix; returns a dict of booleans and figures."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    diag_err = float(np.max(np.abs(np.diag(K) - 1.0))) if n else 0.0
    sym_err = float(np.max(np.abs(K - K.T))) if n else 0.0
    lo = float(K.min()) if n else 0.0
    hi = float(K.max()) if n else 0.0
    lam_min = float(np.linalg.eigvalsh(0.5 * (K + K.T)).min()) if n else 0.0
    if psd_tol is None:
        psd_tol = 1e-8 * max(n, 1)
    return {
        "diag_ok": diag_err <= diag_tol, "diag_err": diag_err,
        "sym_ok": sym_err <= sym_tol, "sym_err": sym_err,
        "range_ok": lo >= -1e-12 and hi <= 1.0 + 1e-5, "min": lo, "max": hi,
        "psd_ok": lam_min >= -psd_tol, "lambda_min": lam_min,
    }
