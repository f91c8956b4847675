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
