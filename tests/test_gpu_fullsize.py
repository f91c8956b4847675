"""Full-size parity: the 784-qubit image workload (4000 train + 1000 test,
L = 2, chi_max 64) in the launch configuration the benchmark times (one
persistent multi-task sweep with the fused epilogue), checked on the seeded
200-pair subset stored by tests/golden/make_golden.py (exact path-sum
values) and by properties that hold at any size."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks  # noqa: E402
from synthdata import config_inputs  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("prec,ln_tol", [("auto", 1e-3), ("fp64", 1e-3), ("fp32_mfma", 1e-3),
                                         ("bf16x3", 1e-3), ("bf16x2", 1e-2)])
def test_c3_full_gram_sampled(prec, ln_tol):
    """Every form meets gate A (entries near 1 are FP64-refined) and gate B,
    except BF16x2, whose 2^-17 products leave |d ln K_q| up to ~5e-3 after
    784 sites: it is held to 1e-2 and is never chosen for such depths."""
    import paper_2602_01330_amd.qk as qk
    g = json.load(open(os.path.join(GOLDEN, "c3_pathsum_200.json")))
    x_tr, x_te, _ = config_inputs("C3")
    print(f"[C3 full {prec}] 4000+1000 d=784", flush=True)
    dev = torch.device("cuda")
    xtr = torch.as_tensor(x_tr, device=dev)
    xte = torch.as_tensor(x_te, device=dev)
    store = qk.QK_STORE_FP64 if prec == "fp64" else qk.QK_STORE_ALL
    btr = qk.qk_mps_build(xtr, 2, 64, 1e-10, store=store)
    bte = qk.qk_mps_build(xte, 2, 64, 1e-10, store=store)
    f64 = dict(dtype=torch.float64, device=dev)
    A = {k: torch.full((4000, 4000), float("nan"), **f64) for k in ("kq", "ln", "kc", "k")}
    B = {k: torch.full((1000, 4000), float("nan"), **f64) for k in ("kq", "ln", "kc", "k")}
    tasks = [
        {"rows": btr, "cols": btr, "symmetric": True, "kq": A["kq"], "lnkq": A["ln"],
         "fuse": {"x_rows": xtr, "x_cols": xtr, "gamma": 1 / 784, "w": 0.5, "kc": A["kc"],
                  "k": A["k"]}},
        {"rows": bte, "cols": btr, "symmetric": False, "kq": B["kq"], "lnkq": B["ln"],
         "fuse": {"x_rows": xte, "x_cols": xtr, "gamma": 1 / 784, "w": 0.5, "kc": B["kc"],
                  "k": B["k"]}},
    ]
    qk.qk_overlap_gram_multi(tasks, prec)
    torch.cuda.synchronize()
    info = qk.qk_mps_info(btr)
    qk.qk_mps_info(bte)
    assert info["chi_realized_max"] == 4 and info["chi_pad"] == 4
    pick = lambda M, rs: (A if rs == 0 else B)[M]
    got = {k: np.array([pick(k, rs)[i, j].item() for rs, i, j in g["pairs"]])
           for k in ("kq", "ln", "kc", "k")}
    ok_b, lmax = checks.gate_b(got["ln"], np.array(g["lnkq"]), tol=ln_tol)
    print(f"[C3 full {prec}] max |d lnK| on the subset = {lmax:.3e}", flush=True)
    assert ok_b, lmax
    for key, ref in (("kq", "kq"), ("kc", "kc"), ("k", "k_w0.5")):
        ok, dmax, rel = checks.gate_a(got[key], np.array(g[ref]))
        assert ok, (key, dmax, rel)
    # properties at full size
    kq = A["kq"].cpu().numpy()
    assert np.all(np.isfinite(kq)) and np.all(np.isfinite(B["kq"].cpu().numpy()))
    assert np.max(np.abs(np.diag(kq) - 1.0)) <= 1e-5
    assert np.array_equal(kq, kq.T)
    assert kq.min() >= 0.0 and kq.max() <= 1.0 + 1e-5
    kc = A["kc"].cpu().numpy()
    assert np.array_equal(np.diag(kc), np.ones(4000))


def test_chi64_sweep_784_sites_sampled():
    """The sweep at the truncating regime's full shape: 784 sites with every
    interior bond at 64 (random left-canonical MPS, 4 row and 8 column
    samples). The matrix-core FP32 form and the FP64 form against the
    oracle's sweep on sampled pairs; the symmetric block's diagonal is 1
    (FP64-refined) and the rectangular block is bitwise the same as the
    matching entries of a launch that also holds other pairs."""
    import paper_2602_01330_amd.qk as qk
    from oracle import mps
    from synthdata import gen_isometry_mps
    from tests._util import import_layout_to_oracle

    print("[chi64 784] generating", flush=True)
    cr, tr = gen_isometry_mps(4, 784, 64, seed=31)
    cc, tc = gen_isometry_mps(8, 784, 64, seed=32)
    br = qk.qk_mps_import(cr, tr, 8, 64)
    bc = qk.qk_mps_import(cc, tc, 8, 64)
    f64 = dict(dtype=torch.float64, device="cuda")
    ln32 = torch.full((4, 8), float("nan"), **f64)
    ln64 = torch.full((4, 8), float("nan"), **f64)
    lns = torch.full((8, 8), float("nan"), **f64)
    print("[chi64 784] sweeping", flush=True)
    qk.qk_overlap_gram(br, bc, False, "fp32_mfma", None, ln32)
    qk.qk_overlap_gram(br, bc, False, "fp64", None, ln64)
    qk.qk_overlap_gram(bc, bc, True, "fp32_mfma", None, lns)
    torch.cuda.synchronize()
    ln32, ln64, lns = ln32.cpu().numpy(), ln64.cpu().numpy(), lns.cpu().numpy()
    assert np.all(np.isfinite(ln32)) and np.all(ln32 < -50)  # distinct random states
    assert np.abs(np.diag(lns)).max() < 1e-8
    pairs = [(0, 0), (1, 5), (2, 3), (3, 7)]
    print("[chi64 784] oracle on 4 pairs", flush=True)
    PA = mps.pad_batch(import_layout_to_oracle(cr, tr))
    PB = mps.pad_batch(import_layout_to_oracle(cc, tc))
    ref = mps.ln_kernel_pairs(PA, PB, pairs)
    got32 = np.array([ln32[i, j] for i, j in pairs])
    got64 = np.array([ln64[i, j] for i, j in pairs])
    print(f"[chi64 784] max |d lnK| fp32_mfma {np.abs(got32 - ref).max():.3e}, "
          f"fp64 {np.abs(got64 - ref).max():.3e}", flush=True)
    assert checks.gate_b(got32, ref, tol=1e-3)[0]
    assert np.abs(got64 - ref).max() < 1e-8
    assert checks.gate_b(ln32, ln64, tol=1e-3)[0]


def test_truncating_regime_784_qubits_vs_replay():
    """The truncating regime at full size: 3 images of 784 features, 8 layers,
    chi_max 64 (bonds would reach 2^8 without the cap). The device build's
    bond tables equal the oracle's step-by-step replay, its complex-FP64
    overlaps meet the stated log gate against the replay's, and its
    per-sample discarded weights equal the replay's (fixture written by
    tests/golden/make_golden.py, which calls only the oracle)."""
    import paper_2602_01330_amd.qk as qk
    fx = json.load(open(os.path.join(GOLDEN, "s1_replay_3.json")))
    x, _, _ = config_inputs("S1", n_train=3, n_test=0)
    print("[S1 full] 3 images, d=784, L=8, chi_max=64: building", flush=True)
    xd = torch.as_tensor(x, device="cuda")
    b = qk.qk_mps_build(xd, 8, 64, 1e-10)
    info = qk.qk_mps_info(b)
    assert info["chi_pad"] == 64 and info["chi_realized_max"] == 64
    assert np.array_equal(qk.qk_mps_chi(b), np.array(fx["chi"], dtype=np.int32))
    ln = torch.full((3, 3), float("nan"), dtype=torch.float64, device="cuda")
    qk.qk_overlap_gram(b, b, True, "fp64", None, ln)
    torch.cuda.synchronize()
    ln = ln.cpu().numpy()
    ok, lmax = checks.gate_b(ln, np.array(fx["lnkq"]))
    print(f"[S1 full] max |d lnK| vs replay = {lmax:.3e}", flush=True)
    assert ok, lmax
    assert np.abs(np.diag(ln)).max() < 1e-8
    disc = qk.qk_mps_discarded(b)
    print(f"[S1 full] discarded weight {disc} (replay {fx['discarded']})", flush=True)
    assert np.allclose(disc, fx["discarded"], rtol=1e-6, atol=1e-15)
