"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value:
* hand-worked gate matrices and a hand-derived two-qubit amplitude;
* closed forms of the entangler-free kernel (product of cosines);
* equality of the two definitions in the paper, Eq. (7) vs Eqs. (8)-(10);
* the independent path-sum chain vs brute-force statevectors, and vs the MPS
  route at 784 qubits;
* the exact bond-dimension bound 2^L of this circuit family;
* the truncation error bound (discarded weight) on up to 14 qubits;
* scipy's cdist for the RBF of Eq. (3); the endpoints of Eq. (11);
* Gram-matrix invariants (unit diagonal, symmetry, range, PSD);
* brute-force statevector overlaps of random left-canonical MPS (bonds up
  to 8, not made by the circuit).
"""
import math

import numpy as np
import pytest

from oracle import checks, circuit, classical, closed_form, mps, pathsum
from oracle import statevector as sv
from synthdata import config_inputs, gen_clusters, gen_isometry_mps
from tests._util import import_layout_to_oracle


def _rand(n, seed):
    return np.random.default_rng(seed).uniform(0.0, math.pi, n)


def test_gate_matrices_by_hand():
    # RZ(pi) = diag(-i, i); RZ(0) = I; H^2 = I; RZZ(pi) = diag(-i, i, i, -i).
    assert np.allclose(circuit.rz(math.pi), np.diag([-1j, 1j]))
    assert np.allclose(circuit.rz(0.0), np.eye(2))
    assert np.allclose(circuit.HADAMARD @ circuit.HADAMARD, np.eye(2))
    assert np.allclose(circuit.rzz(math.pi), np.diag([-1j, 1j, 1j, -1j]))
    x = np.array([0.0, 1.0, math.pi])
    assert np.allclose(circuit.rzz_angles(x),
                       [2 * math.pi * (math.pi - 1.0), 0.0])


@pytest.mark.parametrize("L", [1, 2, 3])
def test_entangler_free_closed_forms(L):
    """Statevector and MPS with entanglers off vs per-qubit closed forms."""
    x, y = _rand(5, 10 + L), _rand(5, 20 + L)
    ref = closed_form.kernel_product(x, y, L)
    if L == 1:
        assert closed_form.kernel_L1(x, y) == pytest.approx(ref, rel=1e-12)
    if L == 2:
        assert closed_form.kernel_L2(x, y) == pytest.approx(ref, rel=1e-12)
    assert sv.kernel_overlap(x, y, L, entangle=False) == pytest.approx(ref, rel=1e-11)
    A, _ = mps.build_mps(x, L, 64, entangle=False)
    B, _ = mps.build_mps(y, L, 64, entangle=False)
    ln = mps.ln_kernel_pairs(mps.pad_batch([A]), mps.pad_batch([B]), [(0, 0)])[0]
    assert math.exp(ln) == pytest.approx(ref, rel=1e-11)


def test_two_qubit_amplitude_by_hand():
    """d = 2, L = 1, derived by hand.

    |psi(x)> = 1/2 sum_{s0,s1} exp(-i(x0 s0 + x1 s1) - i theta(x)/2 s0 s1)|s0 s1>,
    so with u = x0 - y0, v = x1 - y1, w = (theta(x) - theta(y))/2:
    <psi(x)|psi(y)> = (e^{iw} cos(u + v) + e^{-iw} cos(u - v)) / 2.
    """
    rng = np.random.default_rng(7)
    for _ in range(5):
        x = rng.uniform(0, math.pi, 2)
        y = rng.uniform(0, math.pi, 2)
        tx = 2 * (math.pi - x[0]) * (math.pi - x[1])
        ty = 2 * (math.pi - y[0]) * (math.pi - y[1])
        u, v, w = x[0] - y[0], x[1] - y[1], 0.5 * (tx - ty)
        a = 0.5 * (np.exp(1j * w) * math.cos(u + v) + np.exp(-1j * w) * math.cos(u - v))
        ref = abs(a) ** 2
        assert sv.kernel_overlap(x, y, 1) == pytest.approx(ref, rel=1e-12)
        A, _ = mps.build_mps(x, 1, 16)
        B, _ = mps.build_mps(y, 1, 16)
        ln = mps.ln_kernel_pairs(mps.pad_batch([A]), mps.pad_batch([B]), [(0, 0)])[0]
        assert math.exp(ln) == pytest.approx(ref, rel=1e-11)
        lnp = pathsum.ln_kernel_pairs(x[None], y[None], 1, [(0, 0)])[0]
        assert math.exp(lnp) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_eq7_equals_compute_uncompute(L):
    """Eq. (7) overlap vs the Eqs. (8)-(10) return amplitude."""
    x, y = _rand(7, 30 + L), _rand(7, 40 + L)
    a = sv.amplitude_compute_uncompute(x, y, L)
    assert abs(a) ** 2 == pytest.approx(sv.kernel_overlap(x, y, L), rel=1e-11)
    # Eq. (9) amplitude is <psi(y)|psi(x)>
    b = np.vdot(sv.state(y, L), sv.state(x, L))
    assert abs(a - b) < 1e-12


@pytest.mark.parametrize("L", [1, 2, 3])
def test_pathsum_vs_statevector(L):
    X = np.stack([_rand(10, 100 + i + 10 * L) for i in range(4)])
    pairs = [(i, j) for i in range(4) for j in range(4)]
    ref = sv.gram(X, X, L)
    ln = pathsum.ln_kernel_pairs(X, X, L, pairs)
    got = np.exp(ln).reshape(4, 4)
    assert np.allclose(got, ref, rtol=1e-10, atol=0)


@pytest.mark.parametrize("L,n", [(1, 9), (2, 10), (3, 8), (2, 1), (2, 2)])
def test_mps_vs_statevector(L, n):
    X = np.stack([_rand(n, 200 + i + 7 * L + n) for i in range(4)])
    M = mps.build_batch(X, L, 64)
    for m, x in zip(M, X):
        # no truncation: the MPS contracts to exactly the statevector
        assert np.allclose(mps.to_state(m), sv.state(x, L).ravel(), atol=1e-9)
    P = mps.pad_batch(M)
    K, LN = mps.gram(P, P)
    ref = sv.gram(X, X, L)
    assert np.allclose(K, ref, rtol=1e-9, atol=1e-14)


def test_mps_vs_pathsum_784_qubits():
    """Full size: 784 qubits, L = 2, image-like inputs, same- and cross-class."""
    x, _, lab = config_inputs("C3", n_train=12, n_test=0)
    M = mps.build_batch(x, 2, 64)
    P = mps.pad_batch(M)
    pairs = [(0, 0), (0, 10), (1, 11), (0, 1), (3, 7), (2, 2)]
    ln_m = mps.ln_kernel_pairs(P, P, pairs)
    ln_p = pathsum.ln_kernel_pairs(x, x, 2, pairs)
    assert np.all(np.abs(ln_m - ln_p) < 1e-6), (ln_m, ln_p)
    # same-class pairs are far larger than cross-class ones (concentration)
    assert ln_m[1] > ln_m[3] + 50


def test_bond_dimension_bound():
    """Each RZZ has operator-Schmidt rank 2 across its own cut only, so the
    exact bond dimension is <= 2^L; for L = 2 the bonds read 2,4,...,4,2."""
    x, _ = gen_clusters(1, 12, 3)
    for L in (1, 2, 3):
        _, chis = mps.build_mps(x[0], L, 64)
        assert max(chis) <= 2 ** L
    _, chis = mps.build_mps(x[0], 2, 64)
    assert chis == [1, 2] + [4] * 9 + [2, 1]
    # a feature at pi zeroes both neighbouring entangler angles
    xx = x[0].copy()
    xx[5] = math.pi
    _, chis = mps.build_mps(xx, 1, 64)
    assert chis[5] == 1 and chis[6] == 1


def test_truncation_error_bound_and_invariants():
    """chi_max below the exact bond dimension: per-sample truncation keeps
    states normalised, and the kernel error is bounded by the discarded
    weight: |K' - K| <= 2 (||a' - a|| + ||b' - b||), ||a' - a||^2 <= 2 sum w."""
    L, n, chi = 5, 12, 6
    X = np.stack([_rand(n, 500 + i) for i in range(5)])
    built = [mps.build_mps(x, L, chi, return_discarded=True) for x in X]
    assert any(b[2] > 1e-8 for b in built)  # truncation really happened
    P = mps.pad_batch([b[0] for b in built])
    K, _ = mps.gram(P, P)
    ref = sv.gram(X, X, L)
    inv = checks.invariants(K)
    assert inv["diag_ok"] and inv["psd_ok"] and inv["range_ok"]
    eps = [math.sqrt(2 * b[2]) for b in built]
    for i in range(5):
        for j in range(5):
            assert abs(K[i, j] - ref[i, j]) <= 2 * (eps[i] + eps[j]) + 1e-12


def test_rbf_vs_cdist():
    from scipy.spatial.distance import cdist
    X, _ = gen_clusters(30, 16, 11)
    Y, _ = gen_clusters(20, 16, 12)
    g = 1.0 / 16
    ref = np.exp(-g * cdist(X, Y, "sqeuclidean"))
    assert np.allclose(classical.rbf_gram(X, Y, g), ref, rtol=1e-13, atol=0)


def test_mix_endpoints_and_linearity():
    rng = np.random.default_rng(3)
    kq, kc = rng.uniform(size=(4, 4)), rng.uniform(size=(4, 4))
    assert np.array_equal(classical.mix(kq, kc, 1.0), kq)
    assert np.array_equal(classical.mix(kq, kc, 0.0), kc)
    assert np.allclose(classical.mix(kq, kc, 0.25), 0.25 * kq + 0.75 * kc)


def test_c1_gram_invariants():
    x, _, _ = config_inputs("C1", n_train=60)
    P = mps.pad_batch(mps.build_batch(x, 1, 16))
    K, _ = mps.gram(P, P, symmetric=True)
    inv = checks.invariants(K)
    assert all(inv[k] for k in ("diag_ok", "sym_ok", "range_ok", "psd_ok")), inv
    kc = classical.rbf_gram(x, x, 1.0 / 8)
    inv = checks.invariants(kc)
    assert inv["diag_ok"] and inv["psd_ok"]


def test_special_cases():
    x = _rand(6, 77)
    # identical inputs -> 1
    A, _ = mps.build_mps(x, 2, 64)
    P = mps.pad_batch([A])
    assert math.exp(mps.ln_kernel_pairs(P, P, [(0, 0)])[0]) == pytest.approx(1.0, abs=1e-13)
    # all features at pi -> every entangler angle is zero -> closed form
    y = np.full(6, math.pi)
    z = x.copy()
    z[:] = math.pi
    z[2] = 0.3
    assert sv.kernel_overlap(y, z, 2) == pytest.approx(
        closed_form.kernel_product(y, z, 2), rel=1e-12)
    # d = 1: no entangler at all
    a, b = np.array([0.4]), np.array([1.3])
    assert sv.kernel_overlap(a, b, 1) == pytest.approx(math.cos(0.9) ** 2, rel=1e-13)


def test_tolerance_gates():
    ref = np.array([1.0, 0.5, 1e-9, 1e-30])
    ok, _, _ = checks.gate_a(ref + 5e-6 * np.array([1, 0, 0, 0]), ref)
    assert ok
    ok, _, _ = checks.gate_a(ref + 2e-5 * np.array([1, 0, 0, 0]), ref)
    assert not ok
    ok, _, _ = checks.gate_a(ref * np.array([1, 1.002, 1, 1]), ref)
    assert not ok
    ok, _ = checks.gate_b(np.log(ref) + 5e-4, np.log(ref))
    assert ok
    ok, _ = checks.gate_b(np.log(ref) + 5e-3, np.log(ref))
    assert not ok
    ok, _ = checks.gate_b(np.array([-np.inf]), np.array([-np.inf]))
    assert ok


def test_sweep_on_random_isometries_vs_statevector():
    """The transfer-matrix sweep (Eqs. (9), (10)) on MPS that no circuit made:
    random left-canonical tensors with bonds 1, 2, 4, 8, ..., 8, 4, 2, 1 over
    11 sites. Each state has unit norm, and every overlap equals
    |<psi_i|psi_j>|^2 of the dense vectors."""
    chi, ten = gen_isometry_mps(5, 11, 8, seed=21)
    M = import_layout_to_oracle(chi, ten)
    V = np.stack([mps.to_state(m) for m in M])
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-12)
    for t in M[0]:  # left-canonical: sum_s A^s dagger A^s = I
        g = np.einsum("lsr,lsq->rq", t.conj(), t)
        assert np.allclose(g, np.eye(t.shape[2]), atol=1e-12)
    P = mps.pad_batch(M)
    K, _ = mps.gram(P, P)
    ref = np.abs(V.conj() @ V.T) ** 2
    assert np.allclose(K, ref, rtol=1e-10, atol=1e-15)
    assert np.allclose(np.diag(K), 1.0, atol=1e-12)


def test_svm_decision_vs_scikit_learn():
    """Eqs. (4), (5) on precomputed kernel rows: the oracle's decision values
    equal scikit-learn's SVC decision_function (a library routine) for a
    binary problem on the dual kernel of two classes of the 8-feature
    clusters, with coef_i = alpha_i y_i placed at the support vectors."""
    from sklearn.svm import SVC
    x, _, lab = config_inputs("C1")
    pick = np.where((lab == 0) | (lab == 1))[0]
    tr, te = pick[:30], pick[30:40]
    P = mps.pad_batch(mps.build_batch(x[pick], 1, 16))
    K, _ = mps.gram(P, P)
    kc = classical.rbf_gram(x[pick], x[pick], 1.0 / 8)
    Kmix = classical.mix(K, kc, 0.5)
    ntr = len(tr)
    y = np.where(lab[tr] == 1, 1, -1)
    svc = SVC(kernel="precomputed", C=10.0).fit(Kmix[:ntr, :ntr], y)
    coef = np.zeros(ntr)
    coef[svc.support_] = svc.dual_coef_[0]
    rows = Kmix[ntr:, :ntr]
    f = classical.svm_decision(rows, coef, float(svc.intercept_[0]))
    assert np.allclose(f, svc.decision_function(rows), rtol=1e-10, atol=1e-12)
    # sign(f) is the predicted label: scikit-learn's classes_ are (-1, +1)
    assert np.array_equal(np.where(f > 0, 1, -1), svc.predict(rows))


def _c1_dual_kernel(n):
    x, _, lab = config_inputs("C1")
    P = mps.pad_batch(mps.build_batch(x[:n], 1, 16))
    K, _ = mps.gram(P, P)
    return classical.mix(K, classical.rbf_gram(x[:n], x[:n], 1.0 / 8), 0.5), lab[:n]


def test_smo_closed_forms():
    """Eqs. (1)-(2) by hand. Identity kernel, labels +1/-1: the equality
    constraint gives a_1 = a_2 = a, the objective a^2 - 2a is least at a = 1
    (b = 0), and C = 0.5 clips it to the bound (b = 0 by symmetry). Linear
    kernel on x = (-2, -1, 1, 2): the hard-margin separator is f(x) = x, so
    the support vectors are +-1 with a = 1/2 and b = 0."""
    from oracle import svm
    a, b, _ = svm.smo(np.eye(2), np.array([1.0, -1.0]), 10.0, 1e-12)
    assert np.array_equal(a, [1.0, 1.0]) and b == 0.0
    a, b, _ = svm.smo(np.eye(2), np.array([1.0, -1.0]), 0.5, 1e-12)
    assert np.array_equal(a, [0.5, 0.5]) and b == 0.0
    X = np.array([-2.0, -1.0, 1.0, 2.0])
    y = np.array([-1.0, -1.0, 1.0, 1.0])
    a, b, _ = svm.smo(np.outer(X, X), y, 100.0, 1e-12)
    assert np.allclose(a, [0.0, 0.5, 0.5, 0.0], atol=1e-12) and abs(b) < 1e-12
    xs = np.linspace(-3, 3, 7)
    f = classical.svm_decision(np.outer(xs, X), a * y, b)
    assert np.allclose(f, xs, atol=1e-12)


def test_smo_kkt_and_scikit_learn_binary():
    """The binary solver on the dual kernel of two classes of the 8-feature
    clusters: feasibility (0 <= a <= C, sum a y = 0), the KKT violation of a
    gradient recomputed from scratch below eps, and the multipliers, bias
    and decision values of scikit-learn's SVC (LIBSVM) at a tight tolerance."""
    from sklearn.svm import SVC

    from oracle import svm
    Km, lab = _c1_dual_kernel(80)
    pick = np.where((lab == 0) | (lab == 1))[0]
    tr, te = pick[:12], pick[12:]
    y = np.where(lab[tr] == 1, 1.0, -1.0)
    Kt = Km[np.ix_(tr, tr)]
    for C in (10.0, 0.05):
        a, b, it = svm.smo(Kt, y, C, 1e-10)
        assert it > 0 and np.all(a >= 0) and np.all(a <= C)
        assert abs(float(np.dot(a, y))) < 1e-12
        G = (np.outer(y, y) * Kt) @ a - 1.0
        v = -y * G
        up = ((y > 0) & (a < C)) | ((y < 0) & (a > 0))
        low = ((y > 0) & (a > 0)) | ((y < 0) & (a < C))
        assert v[up].max() - v[low].min() < 1e-9
        svc = SVC(kernel="precomputed", C=C, tol=1e-12, shrinking=False).fit(Kt, y)
        coef = np.zeros(len(tr))
        coef[svc.support_] = svc.dual_coef_[0]
        assert np.allclose(a * y, coef, atol=1e-7)
        assert abs(b - float(svc.intercept_[0])) < 1e-7
        rows = Km[np.ix_(te, tr)]
        assert np.allclose(classical.svm_decision(rows, a * y, b),
                           svc.decision_function(rows), atol=1e-7)


def test_ovo_voting_vs_scikit_learn():
    """One-against-one over three classes (Section II-B): decision values
    and voted labels equal scikit-learn's SVC with decision_function_shape
    'ovo' (pair order (0,1), (0,2), (1,2); positive means the first class)."""
    from sklearn.svm import SVC

    from oracle import svm
    Km, lab = _c1_dual_kernel(90)
    labs = lab % 3
    coef, b, iters = svm.fit_ovo(Km[:60, :60], labs[:60], 3, C=10.0, eps=1e-10)
    assert np.all(iters > 0)
    assert np.all(coef[0][labs[:60] == 2] == 0.0)  # pair (0, 1) uses no class-2 sample
    svc = SVC(kernel="precomputed", C=10.0, tol=1e-12, shrinking=False,
              decision_function_shape="ovo").fit(Km[:60, :60], labs[:60])
    f, pred = svm.predict_ovo(Km[60:, :60], coef, b, 3)
    assert np.allclose(f, svc.decision_function(Km[60:, :60]), atol=1e-6)
    assert np.array_equal(pred, svc.predict(Km[60:, :60]))


def test_left_out_samples_equal_submatrix_training():
    """A label of -1 leaves a sample out: training on the full matrix with
    the held-out fold masked gives exactly the coefficients, biases and step
    counts of training on the submatrix of the kept samples."""
    from oracle import svm
    Km, lab = _c1_dual_kernel(60)
    labs = lab % 4
    masked = labs.copy()
    masked[20:40] = -1
    keep = np.r_[0:20, 40:60]
    c_full, b_full, it_full = svm.fit_ovo(Km, masked, 4, 10.0, 1e-6)
    c_sub, b_sub, it_sub = svm.fit_ovo(Km[np.ix_(keep, keep)], labs[keep], 4, 10.0, 1e-6)
    assert np.array_equal(c_full[:, keep], c_sub) and np.all(c_full[:, 20:40] == 0.0)
    assert np.array_equal(b_full, b_sub) and np.array_equal(it_full, it_sub)
