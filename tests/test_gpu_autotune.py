"""Autotuner: times the eligible sweep forms on a slice of tiles and makes
QK_PREC_AUTO resolve to the winner; the winner's results meet the gates."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks  # noqa: E402
from synthdata import config_inputs  # noqa: E402
from tests._util import oracle_gram  # noqa: E402

pytestmark = pytest.mark.gpu


def test_autotune_picks_an_eligible_form_and_auto_follows():
    import paper_2602_01330_amd.qk as qk
    x, _, _ = config_inputs("C2", n_train=96)
    b = qk.qk_mps_build(torch.as_tensor(x, device="cuda"), 2, 32)
    form = qk.qk_autotune(b, b, True, max_tiles=64)
    print(f"[autotune] d=64 chi_pad=4 -> {form}", flush=True)
    assert form in ("fp64", "fp32", "fp32_mfma", "bf16x3")
    assert qk.qk_resolve_precision(b, b) == form
    assert any(l.split()[:2] == ["4", "6"] for l in qk.qk_tune_export().splitlines())
    ln = torch.empty((96, 96), dtype=torch.float64, device="cuda")
    qk.qk_overlap_gram(b, b, True, "auto", None, ln)
    torch.cuda.synchronize()
    K, LN = oracle_gram(x, 2, 32, symmetric=True)
    assert checks.gate_b(ln.cpu().numpy(), LN)[0]


def test_tuning_table_carries_the_launch_shape():
    """An exported entry is 'T bucket form wg_per_cu band us_per_tile'; the
    older five-field form still imports (band 4)."""
    import paper_2602_01330_amd.qk as qk
    x, _, _ = config_inputs("C2", n_train=64)
    b = qk.qk_mps_build(torch.as_tensor(x, device="cuda"), 2, 32)
    qk.qk_autotune(b, b, True, max_tiles=16)
    line = [l for l in qk.qk_tune_export().splitlines() if l.split()[:2] == ["4", "6"]][0]
    t = line.split()
    assert len(t) == 6 and int(t[4]) in (2, 4, 8) and int(t[3]) in (1, 2)
    qk.qk_tune_import(f"4 6 {qk.PREC['fp32_mfma']} 2 1.5\n")
    line = [l for l in qk.qk_tune_export().splitlines() if l.split()[:2] == ["4", "6"]][0]
    assert line.split()[2:5] == [str(qk.PREC["fp32_mfma"]), "2", "4"]
    with pytest.raises(qk.QkError):
        qk.qk_tune_import("4 6 5 2 0 1.0\n")  # band must be >= 1
    b.close()


def test_launch_shapes_give_bitwise_equal_results():
    """The launch shapes the autotuner chooses between (one or two
    workgroups per CU, band heights 2, 4, 8 of the tile order) change only
    which workgroup computes which tile: every
    output of the FP32 matrix-core form (with its FP64 refinement) is
    bitwise the same for all of them, on a symmetric 200-sample task with a
    ragged edge plus a 37 x 200 rectangle in the same launch, and meets the
    gates against the oracle."""
    import paper_2602_01330_amd.qk as qk
    x, xt, _ = config_inputs("C2", n_train=200, n_test=37)
    xd, xtd = torch.as_tensor(x, device="cuda"), torch.as_tensor(xt, device="cuda")
    b, bt = qk.qk_mps_build_many([xd, xtd], 2, 32)
    saved = [l for l in qk.qk_tune_export().splitlines() if l.split()[:2] == ["4", "6"]]
    outs = {}
    try:
        for wg in (2, 1):
            for band in (2, 4, 8):
                qk.qk_tune_import(f"4 6 {qk.PREC['fp32_mfma']} {wg} {band} 1.0\n")
                f64 = dict(dtype=torch.float64, device="cuda")
                ln = torch.full((200, 200), float("nan"), **f64)
                k = torch.full((200, 200), float("nan"), **f64)
                ln2 = torch.full((37, 200), float("nan"), **f64)
                qk.qk_overlap_gram_multi(
                    [{"rows": b, "cols": b, "symmetric": True, "lnkq": ln,
                      "fuse": {"x_rows": xd, "x_cols": xd, "gamma": 1 / 64, "w": 0.5, "k": k}},
                     {"rows": bt, "cols": b, "symmetric": False, "lnkq": ln2}], "fp32_mfma")
                torch.cuda.synchronize()
                outs[(wg, band)] = [t.cpu().numpy() for t in (ln, k, ln2)]
                print(f"[launch shapes] wg={wg} band={band} done", flush=True)
    finally:
        qk.qk_tune_import("\n".join(saved) + "\n" if saved
                          else f"4 6 {qk.PREC['fp32_mfma']} 2 4 0\n")
    ref = outs[(2, 4)]
    for key, v in outs.items():
        for a, r in zip(v, ref):
            assert np.array_equal(a, r), key
    K, LN = oracle_gram(x, 2, 32, symmetric=True)
    assert checks.gate_b(ref[0], LN)[0]
    _, LN2 = oracle_gram(xt, 2, 32, Y=x)
    assert checks.gate_b(ref[2], LN2)[0]
    b.close()
    bt.close()
