"""Full-size parity of the 64-feature cluster workload (2000 train + 500
test samples, L = 2, chi_max 32, cutoff 1e-10) in the launch the benchmark
uses (one multi-task call with the fused RBF and mix), for the chosen form
(AUTO) and the plain complex-FP64 sweep:

- 400 seeded pairs (40 on the diagonal, 120 test x train) against the
  oracle's exact path-sum (ln K_q, gate B; K_q, K_c, K, gate A);
- properties of the full matrices: unit diagonal, exact symmetry, range,
  and positive semidefiniteness (eigvalsh of the 2000 x 2000 K_q, K_c, K:
  lambda_min >= -N max|dK| by Weyl's inequality, with max|dK| <= 1e-5 from
  gate A, against the exact Gram matrices of Eqs. (7), (3), (11), which
  are PSD).
Also: the 784-qubit image workload's full 4000 x 4000 matrices are PSD in
the same sense, and SVM training of problems above 256 samples (the solver
kernel's per-thread sample loops) is bit-identical to the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, classical, mps  # noqa: E402
from oracle import pathsum as opath  # noqa: E402
from synthdata import config_inputs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qk():
    import paper_2602_01330_amd.qk as qk
    return qk


@pytest.fixture(scope="module")
def c2():
    x_tr, x_te, _ = config_inputs("C2")
    rng = np.random.default_rng(2024)
    diag = rng.choice(2000, 40, replace=False)
    tri = rng.integers(0, 2000, size=(240, 2))
    te = np.stack([rng.integers(0, 500, 120), rng.integers(0, 2000, 120)], axis=1)
    pairs_tr = np.concatenate([np.stack([diag, diag], 1), tri])
    ln_tr = opath.ln_kernel_pairs(x_tr, x_tr, 2, pairs_tr)
    ln_te = opath.ln_kernel_pairs(x_te, x_tr, 2, te)
    return x_tr, x_te, pairs_tr, te, ln_tr, ln_te


def lam_min(K):
    return float(np.linalg.eigvalsh(0.5 * (K + K.T)).min())


@pytest.mark.parametrize("prec", ["auto", "fp64"])
def test_c2_full_size(qk, c2, prec):
    x_tr, x_te, pairs_tr, pairs_te, ln_tr, ln_te = c2
    d, n = 64, 2000
    print(f"[C2 full {prec}] 2000 + 500, d=64, L=2, chi_max 32", flush=True)
    xtr = torch.as_tensor(x_tr, device="cuda")
    xte = torch.as_tensor(x_te, device="cuda")
    btr, bte = qk.qk_mps_build_many([xtr, xte], 2, 32, 1e-10)
    f64 = dict(dtype=torch.float64, device="cuda")
    A = {k: torch.full((n, n), float("nan"), **f64) for k in ("kq", "ln", "kc", "k")}
    B = {k: torch.full((500, n), float("nan"), **f64) for k in ("kq", "ln", "kc", "k")}
    tasks = [{"rows": btr, "cols": btr, "symmetric": True, "kq": A["kq"], "lnkq": A["ln"],
              "fuse": {"x_rows": xtr, "x_cols": xtr, "gamma": 1 / d, "w": 0.5, "kc": A["kc"],
                       "k": A["k"]}},
             {"rows": bte, "cols": btr, "symmetric": False, "kq": B["kq"], "lnkq": B["ln"],
              "fuse": {"x_rows": xte, "x_cols": xtr, "gamma": 1 / d, "w": 0.5, "kc": B["kc"],
                       "k": B["k"]}}]
    qk.qk_overlap_gram_multi(tasks, prec)
    torch.cuda.synchronize()
    info = qk.qk_mps_info(btr)
    assert info["chi_realized_max"] == 4
    a = {k: v.cpu().numpy() for k, v in A.items()}
    b = {k: v.cpu().numpy() for k, v in B.items()}
    # sampled pairs against the exact path-sum
    got = np.concatenate([a["ln"][pairs_tr[:, 0], pairs_tr[:, 1]],
                          b["ln"][pairs_te[:, 0], pairs_te[:, 1]]])
    ref = np.concatenate([ln_tr, ln_te])
    ok, lmax = checks.gate_b(got, ref)
    print(f"[C2 full {prec}] max |d lnK| on 400 pairs = {lmax:.3e}", flush=True)
    assert ok, lmax
    kq_ref = np.exp(ref)
    kc_ref = np.concatenate([
        np.exp(-np.sum((x_tr[pairs_tr[:, 0]] - x_tr[pairs_tr[:, 1]]) ** 2, 1) / d),
        np.exp(-np.sum((x_te[pairs_te[:, 0]] - x_tr[pairs_te[:, 1]]) ** 2, 1) / d)])
    for key, r in (("kq", kq_ref), ("kc", kc_ref), ("k", 0.5 * kq_ref + 0.5 * kc_ref)):
        g = np.concatenate([a[key][pairs_tr[:, 0], pairs_tr[:, 1]],
                            b[key][pairs_te[:, 0], pairs_te[:, 1]]])
        okA, dmax, rel = checks.gate_a(g, r)
        assert okA, (key, dmax, rel)
    # full-matrix properties
    for key in ("kq", "kc", "k", "ln"):
        assert np.all(np.isfinite(a[key])) and np.all(np.isfinite(b[key]))
        assert np.array_equal(a[key], a[key].T), key
    assert np.max(np.abs(np.diag(a["kq"]) - 1.0)) <= 1e-5
    assert np.array_equal(np.diag(a["kc"]), np.ones(n))
    for key in ("kq", "kc", "k"):
        assert a[key].min() >= -1e-12 and a[key].max() <= 1.0 + 1e-5
        assert b[key].min() >= -1e-12 and b[key].max() <= 1.0 + 1e-5
        lm = lam_min(a[key])
        print(f"[C2 full {prec}] lambda_min({key}) = {lm:.4e}", flush=True)
        assert lm >= -n * 1e-5, (key, lm)
    # every off-diagonal K_q is far below 1e-8 here, so K_q is the identity
    # to within 1e-8 and its spectrum sits at 1
    assert lam_min(a["kq"]) > 0.99
    for bb in (btr, bte):
        bb.close()


def test_c3_full_matrices_are_psd(qk):
    """The 784-qubit image workload (4000 train, L = 2, chi_max 64) under
    AUTO: the full symmetric K_q, K_c and K have lambda_min >= -N max|dK|
    (eigvalsh of 4000 x 4000)."""
    x_tr, _, _ = config_inputs("C3", n_test=0)
    n, d = x_tr.shape
    print("[C3 psd] 4000 train, d=784", flush=True)
    xtr = torch.as_tensor(x_tr, device="cuda")
    b = qk.qk_mps_build(xtr, 2, 64, 1e-10)
    f64 = dict(dtype=torch.float64, device="cuda")
    kq, kc, k = (torch.full((n, n), float("nan"), **f64) for _ in range(3))
    qk.qk_overlap_gram(b, b, True, "auto", kq, None,
                       {"x_rows": xtr, "x_cols": xtr, "gamma": 1 / d, "w": 0.5, "kc": kc, "k": k})
    torch.cuda.synchronize()
    for key, m in (("kq", kq), ("kc", kc), ("k", k)):
        M = m.cpu().numpy()
        assert np.array_equal(M, M.T)
        lm = lam_min(M)
        print(f"[C3 psd] lambda_min({key}) = {lm:.4e}", flush=True)
        assert lm >= -n * 1e-5, (key, lm)
    b.close()


@pytest.mark.parametrize("n_per_class,n_classes", [(150, 10), (560, 2)])
def test_svm_fit_above_256_samples_per_problem(qk, n_per_class, n_classes):
    """SMO training (Eqs. (1)-(2)) on problems of 300 and 1120 samples: the
    solver kernel's 256-thread workgroup walks each problem's samples in
    strides of 256, so these sizes take 2 and 5 passes per step. The kernel
    matrix is the oracle's (shared by both sides, FP64): step counts,
    multipliers and biases bit-identical to the oracle's, decision values
    to rounding, votes equal."""
    from oracle import svm
    n = n_per_class * n_classes
    x, _, lab = config_inputs("C1", n_train=n + 64)
    lab = lab % n_classes
    P = mps.pad_batch(mps.build_batch(x, 1, 16))
    K, _ = mps.gram(P, P)
    Km = classical.mix(K, classical.rbf_gram(x, x, 1.0 / 8), 0.5)
    Ktr, Kte, ltr = Km[:n, :n].copy(), Km[n:, :n].copy(), lab[:n]
    print(f"[svm large] {n_classes} classes x {n_per_class}: problems of "
          f"{2 * n_per_class} samples", flush=True)
    kd = torch.as_tensor(Ktr, device="cuda")
    coef, b, it = qk.qk_svm_fit_ovo(kd, ltr, n_classes, 1.0, 1e-3)
    torch.cuda.synchronize()
    c_ref, b_ref, it_ref = svm.fit_ovo(Ktr, ltr, n_classes, 1.0, 1e-3)
    print(f"[svm large] steps {it.cpu().numpy().max()} (oracle {it_ref.max()})", flush=True)
    assert np.array_equal(it.cpu().numpy(), it_ref)
    assert np.array_equal(coef.cpu().numpy(), c_ref)
    assert np.array_equal(b.cpu().numpy(), b_ref)
    f, pred = qk.qk_svm_predict_ovo(torch.as_tensor(Kte, device="cuda"), coef, b, n_classes)
    torch.cuda.synchronize()
    f_ref, pred_ref = svm.predict_ovo(Kte, c_ref, b_ref, n_classes)
    assert np.allclose(f.cpu().numpy(), f_ref, rtol=1e-12, atol=1e-12)
    clear = np.min(np.abs(f_ref), axis=1) > 1e-9
    assert np.array_equal(pred.cpu().numpy()[clear], pred_ref[clear])
