"""Block-structured entanglers on the device (Section II-C's block product
state circuits: the RZZ chain restricted to blocks of B consecutive qubits):
the device build's bond tables equal the oracle's (1 at every block
boundary), its overlaps meet the stated gates against the oracle's MPS route
and the exact path-sum, for the FP64 and the chosen forms, at bond bounds 2,
4 and 16 (tile and per-pair sweeps); the device path-sum takes the same
blocks."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, mps  # noqa: E402
from oracle import pathsum as opath  # noqa: E402
from synthdata import config_inputs, gen_clusters  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qk():
    import paper_2602_01330_amd.qk as qk
    return qk


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("d,L,B,T", [(64, 2, 2, 2), (64, 2, 4, 4), (63, 2, 5, 4), (40, 4, 8, 16)])
@pytest.mark.parametrize("prec", ["fp64", "auto", "fp32_mfma"])
def test_block_circuits_against_the_oracle(qk, d, L, B, T, prec):
    X, _ = gen_clusters(24, d, 1200 + d + B)
    Y, _ = gen_clusters(7, d, 1300 + d + B)
    print(f"[blocks] d={d} L={L} B={B} prec={prec}", flush=True)
    xd, yd = dev(X), dev(Y)
    bx = qk.qk_mps_build(xd, L, 64, 1e-10, entangle=B)
    by = qk.qk_mps_build(yd, L, 64, 1e-10, entangle=B)
    info = qk.qk_mps_info(bx)
    assert info["chi_pad"] == T
    chi = qk.qk_mps_chi(bx)
    ref_chi = np.array([mps.build_mps(x, L, 64, 1e-10, entangle=B)[1] for x in X], dtype=np.int32)
    assert np.array_equal(chi, ref_chi)
    assert np.all(chi[:, B::B] == 1)  # every block boundary
    f64 = dict(dtype=torch.float64, device="cuda")
    kq = torch.full((24, 24), float("nan"), **f64)
    ln = torch.full((24, 24), float("nan"), **f64)
    k = torch.full((24, 24), float("nan"), **f64)
    qk.qk_overlap_gram(bx, bx, True, prec, kq, ln,
                       {"x_rows": xd, "x_cols": xd, "gamma": 1 / d, "w": 0.5, "k": k})
    ln2 = torch.full((7, 24), float("nan"), **f64)
    qk.qk_overlap_gram(by, bx, False, prec, None, ln2)
    torch.cuda.synchronize()
    P = mps.pad_batch(mps.build_batch(X, L, 64, 1e-10, entangle=B))
    Q = mps.pad_batch(mps.build_batch(Y, L, 64, 1e-10, entangle=B))
    K, LN = mps.gram(P, P, symmetric=True)
    _, LN2 = mps.gram(Q, P)
    ok_a, dmax, rel = checks.gate_a(kq.cpu().numpy(), K)
    ok_b, lmax = checks.gate_b(ln.cpu().numpy(), LN)
    ok_b2, lmax2 = checks.gate_b(ln2.cpu().numpy(), LN2)
    print(f"[blocks] max|dK| {dmax:.2e} max|dlnK| {lmax:.2e} / {lmax2:.2e}", flush=True)
    assert ok_a and ok_b and ok_b2, (dmax, rel, lmax, lmax2)
    if prec == "fp64":
        assert lmax < 1e-8 and lmax2 < 1e-8
    if L <= 3:  # the exact path-sum with the same blocks
        pairs = [(i, j) for i in range(0, 24, 5) for j in range(24)]
        lref = opath.ln_kernel_pairs(X, X, L, pairs, entangle=B)
        got = np.array([ln[i, j].item() for i, j in pairs])
        assert checks.gate_b(got, lref)[0]
    bx.close()
    by.close()


@pytest.mark.parametrize("B", [3, 16])
def test_block_images_784_sampled(qk, B):
    """The 784-qubit images with entangler blocks of B pixels (L = 2): one
    fused multi-task call in the chosen form, 120 sampled pairs against the
    oracle's exact path-sum with the same blocks."""
    x_tr, x_te, _ = config_inputs("C3", n_train=300, n_test=60)
    print(f"[blocks 784] B={B}", flush=True)
    xtr, xte = dev(x_tr), dev(x_te)
    btr, bte = qk.qk_mps_build_many([xtr, xte], 2, 64, 1e-10, entangle=B)
    chi = qk.qk_mps_chi(btr)
    assert np.all(chi[:, B::B] == 1) and chi.max() == (2 if B < 4 else 4)
    f64 = dict(dtype=torch.float64, device="cuda")
    ln_tr = torch.full((300, 300), float("nan"), **f64)
    ln_te = torch.full((60, 300), float("nan"), **f64)
    qk.qk_overlap_gram_multi([{"rows": btr, "cols": btr, "symmetric": True, "lnkq": ln_tr},
                              {"rows": bte, "cols": btr, "symmetric": False, "lnkq": ln_te}],
                             "auto")
    torch.cuda.synchronize()
    rng = np.random.default_rng(B)
    p_tr = np.concatenate([np.stack([np.arange(20), np.arange(20)], 1),
                           rng.integers(0, 300, size=(60, 2))])
    p_te = np.stack([rng.integers(0, 60, 40), rng.integers(0, 300, 40)], 1)
    ref = np.concatenate([opath.ln_kernel_pairs(x_tr, x_tr, 2, p_tr, entangle=B),
                          opath.ln_kernel_pairs(x_te, x_tr, 2, p_te, entangle=B)])
    got = np.concatenate([ln_tr.cpu().numpy()[p_tr[:, 0], p_tr[:, 1]],
                          ln_te.cpu().numpy()[p_te[:, 0], p_te[:, 1]]])
    ok, lmax = checks.gate_b(got, ref)
    print(f"[blocks 784] max |d lnK| = {lmax:.3e}", flush=True)
    assert ok, lmax
    btr.close()
    bte.close()


@pytest.mark.parametrize("L,B", [(1, 4), (2, 3), (3, 6)])
def test_device_pathsum_with_blocks(qk, L, B):
    X, _ = gen_clusters(33, 30, 1400 + L + B)
    print(f"[blocks pathsum] L={L} B={B}", flush=True)
    xd = dev(X)
    ln = torch.full((33, 33), float("nan"), dtype=torch.float64, device="cuda")
    qk.qk_pathsum_gram(xd, None, L, B, None, ln)
    torch.cuda.synchronize()
    pairs = [(i, j) for i in range(33) for j in range(33)]
    ref = opath.ln_kernel_pairs(X, X, L, pairs, entangle=B).reshape(33, 33)
    assert np.max(np.abs(ln.cpu().numpy() - ref)) < 1e-8
