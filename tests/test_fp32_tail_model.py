"""The host emulation of the reduced-precision sweep (tests/fp32_tail_model.py)
reproduces the oracle's FP64 sweep exactly when run in complex128 (the
rescale every 8 sites is a power of two, hence exact), and in complex64
stays within the single-precision error scale on a short register."""
import numpy as np

from oracle import mps
from synthdata import gen_clusters
from tests.fp32_tail_model import sweep


def test_emulation_matches_the_oracle_sweep_and_single_precision_scale():
    X, _ = gen_clusters(12, 40, 77)
    pad = mps.pad_batch(mps.build_batch(X, 2, 64))
    ia, jb = np.triu_indices(12)
    ref = mps.ln_kernel_pairs(pad, pad, np.stack([ia, jb], 1))
    l64, _ = sweep(pad, ia, jb, np.complex128)
    assert np.allclose(l64, ref, rtol=0, atol=1e-12)
    l32, drops = sweep(pad, ia, jb, np.complex64)
    d = np.abs(l32 - ref)
    assert d.max() < 1e-3 and d.max() > 1e-9  # single precision, not double
    assert (drops >= 0).all()
