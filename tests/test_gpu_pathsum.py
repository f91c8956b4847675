"""The exact path-sum evaluator on the device (circuits of one to three layers).

Checked against the oracle's path-sum (itself pinned to the statevector on
up to 12 qubits and to the MPS oracle at 784 qubits), the entangler-free
closed forms, and the device's own complex-FP64 MPS route on the same
inputs; the fused RBF and mix against the oracle's.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, classical, closed_form, pathsum  # noqa: E402
from synthdata import config_inputs, gen_clusters  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qk():
    import paper_2602_01330_amd.qk as qk
    return qk


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def all_pairs(m, n):
    return np.array([(i, j) for i in range(m) for j in range(n)])


@pytest.mark.parametrize("L", [1, 2, 3])
@pytest.mark.parametrize("m,n", [(37, 37), (17, 33), (1, 1)])
def test_pathsum_vs_oracle(qk, L, m, n):
    """Symmetric (37 samples: three tiles, a ragged edge) and rectangular
    calls against the oracle's path-sum, entry by entry: both FP64 with
    exact rescaling, so ln K agrees to rounding."""
    X, _ = gen_clusters(m, 8, 70 + m + L)
    sym = m == n and m > 1
    Y = X if sym else gen_clusters(n, 8, 90 + n + L)[0]
    print(f"[pathsum] L={L} {m}x{n} sym={sym}", flush=True)
    ln = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    kq = torch.full((m, n), float("nan"), dtype=torch.float64, device="cuda")
    xr = dev(X)
    qk.qk_pathsum_gram(xr, None if sym else dev(Y), L, True, kq, ln)
    torch.cuda.synchronize()
    ref = pathsum.ln_kernel_pairs(X, Y, L, all_pairs(m, n)).reshape(m, n)
    got = ln.cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-11
    assert np.allclose(kq.cpu().numpy(), np.exp(ref), rtol=1e-10, atol=0)
    if sym:
        assert np.array_equal(got, got.T)
        assert np.max(np.abs(np.diag(got))) < 1e-12


@pytest.mark.parametrize("L", [1, 2, 3])
def test_pathsum_without_entanglers_is_the_product_form(qk, L):
    """entangle = 0: the kernel is the product of per-qubit overlaps (closed
    form, no chain)."""
    X, _ = gen_clusters(20, 16, 5 + L)
    kq = torch.empty((20, 20), dtype=torch.float64, device="cuda")
    qk.qk_pathsum_gram(dev(X), None, L, False, kq, None)
    torch.cuda.synchronize()
    ref = np.array([[closed_form.kernel_product(a, b, L) for b in X] for a in X])
    assert np.allclose(kq.cpu().numpy(), ref, rtol=1e-11, atol=1e-300)


def test_pathsum_equals_mps_route_at_784_qubits(qk):
    """The 784-feature images at L = 2: the path-sum and the device's
    complex-FP64 MPS sweep (cutoff 1e-10, bonds 4, no truncation) give the
    same ln K_q, train x train and test x train; sampled pairs also match the
    oracle's path-sum; the fused RBF and mix match the oracle's."""
    x_tr, x_te, _ = config_inputs("C3", n_train=40, n_test=20)
    xtr, xte = dev(x_tr), dev(x_te)
    print("[pathsum 784] 40 train + 20 test", flush=True)
    f64 = dict(dtype=torch.float64, device="cuda")
    ln_ps = torch.empty((40, 40), **f64)
    ln_te = torch.empty((20, 40), **f64)
    kc = torch.empty((20, 40), **f64)
    k = torch.empty((20, 40), **f64)
    qk.qk_pathsum_gram(xtr, None, 2, True, None, ln_ps)
    qk.qk_pathsum_gram(xte, xtr, 2, True, None, ln_te,
                       {"gamma": 1.0 / 784, "w": 0.3, "kc": kc, "k": k})
    b_tr = qk.qk_mps_build(xtr, 2, 64, 1e-10, store=qk.QK_STORE_FP64)
    b_te = qk.qk_mps_build(xte, 2, 64, 1e-10, store=qk.QK_STORE_FP64)
    ln_m = torch.empty((40, 40), **f64)
    ln_mt = torch.empty((20, 40), **f64)
    qk.qk_overlap_gram(b_tr, b_tr, True, "fp64", None, ln_m)
    qk.qk_overlap_gram(b_te, b_tr, False, "fp64", None, ln_mt)
    torch.cuda.synchronize()
    d1 = np.max(np.abs(ln_ps.cpu().numpy() - ln_m.cpu().numpy()))
    d2 = np.max(np.abs(ln_te.cpu().numpy() - ln_mt.cpu().numpy()))
    print(f"[pathsum 784] max |d lnK| vs MPS: {d1:.2e} {d2:.2e}", flush=True)
    assert d1 < 1e-8 and d2 < 1e-8
    rng = np.random.default_rng(784)
    pairs = np.stack([rng.integers(0, 20, 60), rng.integers(0, 40, 60)], axis=1)
    ref = pathsum.ln_kernel_pairs(x_te, x_tr, 2, pairs)
    got = ln_te.cpu().numpy()[pairs[:, 0], pairs[:, 1]]
    assert np.max(np.abs(got - ref)) < 1e-9
    kc_ref = classical.rbf_gram(x_te, x_tr, 1.0 / 784)
    assert np.allclose(kc.cpu().numpy(), kc_ref, rtol=1e-13, atol=0)
    K_ref = classical.mix(np.exp(ln_te.cpu().numpy()), kc_ref, 0.3)
    assert checks.gate_a(k.cpu().numpy(), K_ref)[0]
    b_tr.close()
    b_te.close()


def test_pathsum_rejections(qk):
    X, _ = gen_clusters(4, 6, 1)
    ln = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(qk.QkError):
        qk.qk_pathsum_gram(dev(X), None, 4, True, None, ln)  # four layers
    with pytest.raises(qk.QkError):
        qk.qk_pathsum_gram(dev(X), None, 2, True, None, None)  # no output
    with pytest.raises(ValueError):
        qk.qk_pathsum_gram(dev(X), dev(X[:, :5]), 2, True, None, ln)
    assert math.isfinite(float(qk.qk_pathsum_gram(dev(X), None, 2, True, None, ln)[1][0, 0]))


def test_pathsum_three_layers_equals_bond8_mps_route(qk):
    """L = 3 at 64 features: bonds reach 8, so the MPS route runs the
    one-workgroup-per-pair complex-FP64 sweep; the path-sum (32 states) gives
    the same ln K_q."""
    X, _ = gen_clusters(24, 64, 364)
    xd = dev(X)
    print("[pathsum L=3] 24 samples, d=64", flush=True)
    ln_ps = torch.empty((24, 24), dtype=torch.float64, device="cuda")
    qk.qk_pathsum_gram(xd, None, 3, True, None, ln_ps)
    b = qk.qk_mps_build(xd, 3, 64, 1e-10, store=qk.QK_STORE_FP64)
    assert qk.qk_mps_info(b)["chi_pad"] == 8
    ln_m = torch.empty((24, 24), dtype=torch.float64, device="cuda")
    qk.qk_overlap_gram(b, b, True, "fp64", None, ln_m)
    torch.cuda.synchronize()
    assert np.max(np.abs(ln_ps.cpu().numpy() - ln_m.cpu().numpy())) < 1e-8
    b.close()
