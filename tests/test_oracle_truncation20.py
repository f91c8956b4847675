"""The truncating schedule of the 784-qubit, 8-layer workload (chi_max 64,
relative cutoff 1e-10, renormalised per sample) on registers small enough
for a statevector: 20 qubits, where the exact bond reaches 2^10, so the cap
binds in the middle of the chain. The exact kernel comes from dense
statevectors (a construction independent of the MPS code), and the oracle's
truncated MPS kernel must stay within the bound that its own discarded
weights give: |K' - K| <= 2 (||a' - a|| + ||b' - b||) with
||a' - a||^2 <= 2 sum_w. A smaller cap (16) makes the truncation large
enough that the bound is tested with room to fail."""
import math

import numpy as np
import pytest

from oracle import checks, mps
from oracle import statevector as sv
from synthdata import gen_clusters


@pytest.mark.parametrize("chi_max", [16, 64])
def test_eight_layer_truncation_at_20_qubits(chi_max):
    X, _ = gen_clusters(4, 20, 6100 + chi_max)
    built = [mps.build_mps(x, 8, chi_max, 1e-10, return_discarded=True) for x in X]
    assert max(max(b[1]) for b in built) == chi_max  # the cap binds
    P = mps.pad_batch([b[0] for b in built])
    K, _ = mps.gram(P, P)
    ref = sv.gram(X, X, 8)
    inv = checks.invariants(K)
    assert inv["diag_ok"] and inv["psd_ok"] and inv["range_ok"] and inv["sym_ok"]
    eps = [math.sqrt(2 * b[2]) for b in built]
    err = np.abs(K - ref)
    bound = 2 * (np.add.outer(eps, eps)) + 1e-12
    assert (err <= bound).all()
    # state level: min over a phase of ||a' - e^{i phi} a||^2 = 2 - 2 |<a|a'>|,
    # at most 2 sum_w for each sample (the tighter form of the same bound)
    gaps = []
    for x, b in zip(X, built):
        ov = abs(np.vdot(sv.state(x, 8), mps.to_state(b[0])))
        gaps.append(2.0 - 2.0 * ov)
        assert gaps[-1] <= 2.0 * b[2] + 1e-12
    if chi_max == 16:
        # the truncation is visible in the states and in the kernel
        assert max(gaps) > 1e-4 and err.max() > 1e-9
