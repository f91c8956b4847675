"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case patches one plausible slip into the oracle -- a flipped phase
sign, a dropped complex conjugate, a transposed operand, a wrong angle index
-- and checks that an independent pin (statevector, path-sum, hand-derived
amplitude) disagrees with the patched oracle. This shows the pins have
teeth; it never touches the GPU path.
"""
import math

import numpy as np
import pytest

from oracle import circuit, mps, pathsum
from oracle import statevector as sv


def _pair(n=8, seed=5):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, math.pi, n), rng.uniform(0, math.pi, n)


def _mps_k(x, y, L=2):
    A, _ = mps.build_mps(x, L, 64)
    B, _ = mps.build_mps(y, L, 64)
    return math.exp(mps.ln_kernel_pairs(mps.pad_batch([A]), mps.pad_batch([B]), [(0, 0)])[0])


def _agree(x, y, L=2):
    k_sv = sv.kernel_overlap(x, y, L)
    k_ps = math.exp(pathsum.ln_kernel_pairs(x[None], y[None], L, [(0, 0)])[0])
    k_mps = _mps_k(x, y, L)
    return abs(k_sv - k_mps) < 1e-9 * k_sv and abs(k_ps - k_mps) < 1e-9 * k_ps


def test_unpatched_oracle_agrees():
    assert _agree(*_pair())


def test_flipped_entangler_sign_is_caught(monkeypatch):
    orig = mps._SIGMA.copy()
    monkeypatch.setattr(mps, "_SIGMA", np.array([1.0, 1.0]))  # drops the ZZ sign
    assert not _agree(*_pair())
    monkeypatch.setattr(mps, "_SIGMA", orig)


def test_dropped_conjugate_in_sweep_is_caught(monkeypatch):
    def bad_overlap(padA, padB, pairs):
        pairs = np.asarray(pairs).reshape(-1, 2)
        E = np.ones((len(pairs), 1, 1), dtype=complex)
        for Ak, Bk in zip(padA, padB):
            a, b = Ak[pairs[:, 0]], Bk[pairs[:, 1]]
            E = sum(a[:, :, s, :].transpose(0, 2, 1) @ (E @ b[:, :, s, :]) for s in range(2))
        return E[:, 0, 0], np.zeros(len(pairs), dtype=np.int64)
    monkeypatch.setattr(mps, "overlap_pairs", bad_overlap)
    assert not _agree(*_pair())


def test_transposed_site_tensor_is_caught(monkeypatch):
    orig = mps.overlap_pairs

    def transposed(padA, padB, pairs):
        padB = [np.ascontiguousarray(t[:, :, ::-1, :]) for t in padB]  # swaps s
        return orig(padA, padB, pairs)
    monkeypatch.setattr(mps, "overlap_pairs", transposed)
    assert not _agree(*_pair())


def test_shifted_angle_index_is_caught(monkeypatch):
    def shifted(x):
        # slip: the second factor uses x_k instead of x_{k+1}
        x = np.asarray(x, dtype=np.float64)
        return 2.0 * (math.pi - x[:-1]) * (math.pi - x[:-1])
    monkeypatch.setattr(circuit, "rzz_angles", shifted)
    monkeypatch.setattr(sv, "rzz_angles", shifted)
    monkeypatch.setattr(mps, "rzz_angles", shifted)
    monkeypatch.setattr(pathsum, "rzz_angles", shifted)
    # all routes share the slip, so only the hand-derived d = 2 amplitude sees it
    rng = np.random.default_rng(1)
    x, y = rng.uniform(0, math.pi, 2), rng.uniform(0, math.pi, 2)
    tx = 2 * (math.pi - x[0]) * (math.pi - x[1])
    ty = 2 * (math.pi - y[0]) * (math.pi - y[1])
    u, v, w = x[0] - y[0], x[1] - y[1], 0.5 * (tx - ty)
    ref = abs(0.5 * (np.exp(1j * w) * math.cos(u + v) + np.exp(-1j * w) * math.cos(u - v))) ** 2
    assert sv.kernel_overlap(x, y, 1) != pytest.approx(ref, rel=1e-6)


def _svm_vs_libsvm():
    """True when the oracle's OvO decision values match scikit-learn's."""
    from sklearn.svm import SVC

    from oracle import classical, svm
    from synthdata import config_inputs
    x, _, lab = config_inputs("C1")
    x, labs = x[:60], lab[:60] % 3
    Km = classical.rbf_gram(x, x, 1.0 / 8)
    coef, b, _ = svm.fit_ovo(Km[:45, :45], labs[:45], 3, C=10.0, eps=1e-10)
    f, _ = svm.predict_ovo(Km[45:, :45], coef, b, 3)
    svc = SVC(kernel="precomputed", C=10.0, tol=1e-12, shrinking=False,
              decision_function_shape="ovo").fit(Km[:45, :45], labs[:45])
    return bool(np.allclose(f, svc.decision_function(Km[45:, :45]), atol=1e-6))


def test_unpatched_svm_oracle_agrees():
    assert _svm_vs_libsvm()


def test_flipped_svm_bias_sign_is_caught(monkeypatch):
    from oracle import svm
    orig = svm.intercept
    monkeypatch.setattr(svm, "intercept", lambda *a: -orig(*a))
    assert not _svm_vs_libsvm()


def test_swapped_ovo_orientation_is_caught(monkeypatch):
    from oracle import svm
    orig = svm.ovo_pairs
    monkeypatch.setattr(svm, "ovo_pairs", lambda n: [(b, a) for a, b in orig(n)])
    assert not _svm_vs_libsvm()
