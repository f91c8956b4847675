"""Uneven batched sweep: ten feature dimensions d in {2, 4, ..., 784} (one
qubit per feature, 1000 cluster samples each, L = 2, chi_max = min(2^(d/2),
64)) in ONE persistent launch, checked per d on sampled pairs against the
exact path-sum oracle (any qubit count, no MPS)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import checks, pathsum  # noqa: E402
from synthdata import config_inputs  # noqa: E402
from synthdata.generators import C4_DIMS, chi_cap  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["auto", "fp64"])
def test_ten_dims_one_launch(prec):
    import paper_2602_01330_amd.qk as qk
    dev = torch.device("cuda")
    xs, batches, outs, tasks = {}, {}, {}, []
    for d in C4_DIMS:
        x, _, _ = config_inputs("C4", d=d, n_train=1000, n_test=0)
        xs[d] = x
        xd = torch.as_tensor(x, device=dev)
        batches[d] = qk.qk_mps_build(xd, 2, chi_cap("C4", d))
        outs[d] = torch.full((1000, 1000), float("nan"), dtype=torch.float64, device=dev)
        tasks.append({"rows": batches[d], "cols": batches[d], "symmetric": True,
                      "lnkq": outs[d]})
    print(f"[C4 {prec}] one launch, {len(tasks)} tasks", flush=True)
    qk.qk_overlap_gram_multi(tasks, prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    for d in C4_DIMS:
        info = qk.qk_mps_info(batches[d])
        assert info["chi_pad"] == (2 if d == 2 else 4)
        ln = outs[d].cpu().numpy()
        assert np.all(np.isfinite(ln)) and np.array_equal(ln, ln.T)
        pairs = [(i, i) for i in rng.choice(1000, 4, replace=False)]
        pairs += [tuple(rng.choice(1000, 2, replace=False)) for _ in range(16)]
        pairs += [(i, i + 10) for i in rng.choice(990, 6, replace=False)]  # same class
        ref = pathsum.ln_kernel_pairs(xs[d], xs[d], 2, pairs)
        got = np.array([ln[i, j] for i, j in pairs])
        ok_b, lmax = checks.gate_b(got, ref)
        ok_a, dmax, rel = checks.gate_a(np.exp(got), np.exp(ref))
        print(f"[C4 {prec}] d={d}: max |d lnK| {lmax:.2e}, max |dK| {dmax:.2e}", flush=True)
        assert ok_a and ok_b, (d, lmax, dmax, rel)
