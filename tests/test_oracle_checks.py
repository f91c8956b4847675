"""Negative pins of the oracle's Gram-matrix checks: matrices built by hand
so that exactly one invariant is broken must fail that invariant and pass
the others, so a check that always passed would fail here. The kernel of
Eq. (7) is a Gram matrix of unit vectors (unit diagonal, symmetric, values
in [0, 1], positive semidefinite); Eq. (3) shares those properties."""
import math

import numpy as np

from oracle import checks


def flags(K, **kw):
    inv = checks.invariants(K, **kw)
    return {k: inv[k] for k in ("diag_ok", "sym_ok", "range_ok", "psd_ok")}, inv


def test_a_gram_matrix_of_unit_vectors_passes_every_check():
    rng = np.random.default_rng(3)
    V = rng.standard_normal((7, 5)) + 1j * rng.standard_normal((7, 5))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    K = np.abs(V.conj() @ V.T) ** 2  # |<v_i|v_j>|^2: the Hadamard square of a Gram matrix
    f, _ = flags(K)
    assert all(f.values()), f


def test_off_unit_diagonal_fails_only_the_diagonal_check():
    K = np.eye(4)
    K[2, 2] = 1.0 - 1e-7
    f, inv = flags(K)
    assert f == {"diag_ok": False, "sym_ok": True, "range_ok": True, "psd_ok": True}
    assert math.isclose(inv["diag_err"], 1e-7, rel_tol=1e-6)


def test_asymmetry_fails_only_the_symmetry_check():
    K = np.eye(3)
    K[0, 1], K[1, 0] = 0.25, 0.25 + 1e-9
    f, inv = flags(K)
    assert f == {"diag_ok": True, "sym_ok": False, "range_ok": True, "psd_ok": True}
    assert math.isclose(inv["sym_err"], 1e-9, rel_tol=1e-6)


def test_values_outside_the_unit_interval_fail_the_range_check():
    K = np.eye(3)
    K[0, 2] = K[2, 0] = -1e-6  # below the -1e-12 floor; still PSD (diagonally dominant)
    f, _ = flags(K)
    assert f == {"diag_ok": True, "sym_ok": True, "range_ok": False, "psd_ok": True}
    K = np.eye(3)
    K[0, 0] = 1.0 + 2e-5  # above 1 + 1e-5 (and off the unit diagonal)
    f, _ = flags(K)
    assert not f["range_ok"] and not f["diag_ok"] and f["sym_ok"] and f["psd_ok"]


def test_indefinite_matrix_in_range_fails_only_psd():
    """[[1,1,0],[1,1,1],[0,1,1]] has eigenvalues 1 and 1 +- sqrt(2): unit
    diagonal, symmetric, every entry in [0, 1], yet lambda_min = 1 - sqrt(2)."""
    K = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 1.0]])
    f, inv = flags(K)
    assert f == {"diag_ok": True, "sym_ok": True, "range_ok": True, "psd_ok": False}
    assert math.isclose(inv["lambda_min"], 1.0 - math.sqrt(2.0), rel_tol=1e-12)


def test_psd_tolerance_scales_with_size():
    """A rounding-level negative eigenvalue (-1e-9 at n = 2) passes the default
    tolerance 1e-8 n; -1e-6 does not."""
    for eps, ok in ((1e-9, True), (1e-6, False)):
        c = 1.0 + eps  # eigenvalues 1 +- c of [[1, c], [c, 1]]
        f, inv = flags(np.array([[1.0, c], [c, 1.0]]))
        assert f["psd_ok"] is ok and math.isclose(inv["lambda_min"], -eps, rel_tol=1e-4)
