"""The pre-processing of Section II-A on the device (qk_preproc_fit /
qk_preproc_apply: z-score, PCA to n components by a Jacobi eigensolver,
min-max) against the oracle's, on synthetic 28 x 28 images as raw pixel
intensities; then the whole pipeline of the paper's Fig. 2 on the device
(pre-process -> encode -> dual kernel -> SVM), and a cross-validation that
sweeps the RBF width gamma next to w and C on resident kernel matrices."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, classical, mps  # noqa: E402
from oracle import preprocess as opp  # noqa: E402
from synthdata import gen_images  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qk():
    import paper_2602_01330_amd.qk as qk
    return qk


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def raw_images(n, seed):
    x, lab = gen_images(n, seed)
    return x / np.pi, lab  # pixel intensities in [0, 1]


@pytest.mark.parametrize("n_comp", [2, 16, 64, 784])
def test_fit_and_apply_match_the_oracle(qk, n_comp):
    X, _ = raw_images(600, 51)
    Xt, _ = raw_images(50, 52)
    print(f"[preprocess] 600 x 784 -> {n_comp}", flush=True)
    p = qk.qk_preproc_fit(dev(X), n_comp)
    info = qk.qk_preproc_info(p)
    out = torch.empty((600, n_comp), dtype=torch.float64, device="cuda")
    out_t = torch.empty((50, n_comp), dtype=torch.float64, device="cuda")
    qk.qk_preproc_apply(p, dev(X), out, np.pi)
    qk.qk_preproc_apply(p, dev(Xt), out_t, np.pi)
    torch.cuda.synchronize()
    f = opp.fit(X, n_comp)
    lam = f.eigvals
    print(f"[preprocess] Jacobi sweeps {info['sweeps']}, max |d lambda| "
          f"{np.abs(info['eigvals'] - lam).max():.2e} (lambda_0 {lam[0]:.3e})", flush=True)
    assert np.allclose(info["eigvals"], lam, rtol=0, atol=1e-10 * lam[0])
    ref = opp.transform(f, X, np.pi)
    ref_t = opp.transform(f, Xt, np.pi)
    got, got_t = out.cpu().numpy(), out_t.cpu().numpy()
    # components separated from their neighbours by a clear eigenvalue gap
    # are unique up to the fixed sign; compare those columns tightly and the
    # rest (near-degenerate bulk eigenvectors) only through properties
    gap = np.minimum(np.r_[np.inf, -np.diff(lam)][:n_comp], np.r_[-np.diff(lam), np.inf][:n_comp])
    clear = gap > 1e-6 * lam[0]
    err = np.abs(got - ref)[:, clear].max() if clear.any() else 0.0
    print(f"[preprocess] {clear.sum()} well-separated components, max |d u| {err:.2e}", flush=True)
    assert err < 1e-8
    assert np.abs(got_t - ref_t)[:, clear].max() < 1e-8 if clear.any() else True
    assert np.allclose(got.min(axis=0), 0.0, atol=1e-12) and np.allclose(got.max(axis=0), np.pi)
    p.close()


def test_pipeline_preprocess_encode_kernel_svm(qk):
    """Fig. 2 on the device: raw images -> z-score / PCA (16) / min-max to
    [0, 1] -> MPS encoding (16 qubits, L = 2) -> K_q, K_c (gamma = 1/16),
    K (w = 0.5) -> one-against-one SVM; every stage against the oracle run
    on the oracle's own pre-processed features: features within 1e-9, the
    kernels within the stated gates, decision values within 1e-6."""
    from oracle import svm
    X, lab = raw_images(240, 61)
    Xtr, Xte, ytr = X[:200], X[200:], lab[:200]
    xtr_d, xte_d = dev(Xtr), dev(Xte)
    p = qk.qk_preproc_fit(xtr_d, 16)
    ftr = torch.empty((200, 16), dtype=torch.float64, device="cuda")
    fte = torch.empty((40, 16), dtype=torch.float64, device="cuda")
    qk.qk_preproc_apply(p, xtr_d, ftr, 1.0)
    qk.qk_preproc_apply(p, xte_d, fte, 1.0)
    btr, bte = qk.qk_mps_build_many([ftr, fte], 2, 64)
    f64 = dict(dtype=torch.float64, device="cuda")
    k_tr = torch.empty((200, 200), **f64)
    k_te = torch.empty((40, 200), **f64)
    qk.qk_overlap_gram_multi(
        [{"rows": btr, "cols": btr, "symmetric": True,
          "fuse": {"x_rows": ftr, "x_cols": ftr, "gamma": 1 / 16, "w": 0.5, "k": k_tr}},
         {"rows": bte, "cols": btr, "symmetric": False,
          "fuse": {"x_rows": fte, "x_cols": ftr, "gamma": 1 / 16, "w": 0.5, "k": k_te}}], "auto")
    coef, b, it = qk.qk_svm_fit_ovo(k_tr, ytr, 10, 10.0, 1e-3)
    fdev, pred = qk.qk_svm_predict_ovo(k_te, coef, b, 10)
    torch.cuda.synchronize()
    f = opp.fit(Xtr, 16)
    Ftr, Fte = opp.transform(f, Xtr), opp.transform(f, Xte)
    assert np.abs(ftr.cpu().numpy() - Ftr).max() < 1e-9
    assert np.abs(fte.cpu().numpy() - Fte).max() < 1e-9
    Ptr = mps.pad_batch(mps.build_batch(Ftr, 2, 64))
    Pte = mps.pad_batch(mps.build_batch(Fte, 2, 64))
    Kq_tr, _ = mps.gram(Ptr, Ptr, symmetric=True)
    Kq_te, _ = mps.gram(Pte, Ptr)
    K_tr = classical.mix(Kq_tr, classical.rbf_gram(Ftr, Ftr, 1 / 16), 0.5)
    K_te = classical.mix(Kq_te, classical.rbf_gram(Fte, Ftr, 1 / 16), 0.5)
    assert checks.gate_a(k_tr.cpu().numpy(), K_tr)[0]
    assert checks.gate_a(k_te.cpu().numpy(), K_te)[0]
    c_ref, b_ref, _ = svm.fit_ovo(K_tr, ytr, 10, 10.0, 1e-3)
    f_ref, pred_ref = svm.predict_ovo(K_te, c_ref, b_ref, 10)
    assert np.abs(fdev.cpu().numpy() - f_ref).max() < 1e-6
    clear = np.min(np.abs(f_ref), axis=1) > 1e-6
    assert np.array_equal(pred.cpu().numpy()[clear], pred_ref[clear])
    print(f"[pipeline] test accuracy (synthetic labels) "
          f"{(pred.cpu().numpy() == lab[200:]).mean():.3f}", flush=True)
    for bb in (btr, bte):
        bb.close()
    p.close()


def test_cross_validation_over_gamma_w_and_C(qk):
    """Cross-validation of the dual-kernel SVM over the RBF width gamma (K_c
    recomputed on the device per gamma, Eq. (3)), the mix w (Eq. (11)) and C,
    on resident K_q (3 folds, 5 classes): the device's K_c and mixed K equal
    the oracle's to rounding, and the device trains every fold on the
    oracle's mixed matrix (uploaded) with the oracle's steps, multipliers
    and votes."""
    from oracle import svm
    X, lab = raw_images(120, 71)
    f = opp.fit(X, 8)
    F = opp.transform(f, X, np.pi)
    labs = lab % 5
    P = mps.pad_batch(mps.build_batch(F, 1, 16))
    Kq, _ = mps.gram(P, P)
    fd, kq = dev(F), dev(Kq)
    kc = torch.empty_like(kq)
    k = torch.empty_like(kq)
    folds = [(0, 40), (40, 80), (80, 120)]
    for gamma in (1 / 16, 1 / 8, 1 / 4):
        qk.qk_rbf_gram(fd, fd, gamma, kc)
        torch.cuda.synchronize()
        Kc = classical.rbf_gram(F, F, gamma)
        assert np.abs(kc.cpu().numpy() - Kc).max() < 1e-14
        for w in (0.25, 0.75):
            qk.qk_dual_mix(kq, kc, w, k)
            torch.cuda.synchronize()
            K = classical.mix(Kq, Kc, w)
            assert np.allclose(k.cpu().numpy(), K, rtol=1e-14, atol=1e-14)
            k.copy_(dev(K))  # the solver's input: the oracle's matrix on both sides
            for C_box in (1.0, 10.0):
                for lo, hi in folds:
                    masked = labs.copy()
                    masked[lo:hi] = -1
                    coef, b, it = qk.qk_svm_fit_ovo(k, masked, 5, C_box, 1e-4)
                    _, pred = qk.qk_svm_predict_ovo(k[lo:hi].contiguous(), coef, b, 5)
                    torch.cuda.synchronize()
                    c_ref, b_ref, it_ref = svm.fit_ovo(K, masked, 5, C_box, 1e-4)
                    assert np.array_equal(it.cpu().numpy(), it_ref)
                    assert np.array_equal(coef.cpu().numpy(), c_ref)
                    f_ref, pred_ref = svm.predict_ovo(K[lo:hi], c_ref, b_ref, 5)
                    clear = np.min(np.abs(f_ref), axis=1) > 1e-9
                    assert np.array_equal(pred.cpu().numpy()[clear], pred_ref[clear])
        print(f"[cv] gamma={gamma:.4f}: 12 fits equal the oracle's", flush=True)
