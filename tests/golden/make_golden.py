"""Write the stored expected values under tests/golden/ (calls only oracle/).

* c1_eq7.json: K_q by brute-force statevector, Eq. (7), for every pair of
  the first 24 training samples of the 8-feature, 1-layer cluster workload,
  with K_c (Eq. (3), gamma = 1/d) and K = 0.5 K_q + 0.5 K_c (Eq. (11)).
* c3_pathsum_200.json: ln K_q by the exact path-sum chain for a seeded
  200-pair subset (20 diagonal, 120 train x train, 60 test x train) of the
  784-feature, 2-layer image workload, with K_c and the w = 0.5 mix.
* s1_replay_3.json: the truncating regime at full size (784-feature images,
  seed 6, 8 layers, chi_max 64, cutoff 1e-10): the oracle's step-by-step
  TEBD replay of the first 3 training images (bond tables) and its FP64
  overlaps (ln K_q for every pair, diagonal included).

Run from the repository root: python tests/golden/make_golden.py [s1]
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import classical, mps, pathsum  # noqa: E402
from oracle import statevector as sv  # noqa: E402
from synthdata import config_inputs  # noqa: E402


def c3_subset_pairs(n_train, n_test, seed=2024):
    """Seeded pair subset: (row_set, i, j) with row_set 0 = train, 1 = test."""
    rng = np.random.default_rng(seed)
    diag = rng.choice(n_train, 20, replace=False)
    out = [(0, int(i), int(i)) for i in diag]
    while len(out) < 140:
        i, j = rng.integers(n_train, size=2)
        if i != j:
            out.append((0, int(min(i, j)), int(max(i, j))))
    for _ in range(60):
        out.append((1, int(rng.integers(n_test)), int(rng.integers(n_train))))
    return out


def main():
    x, _, _ = config_inputs("C1")
    x = x[:24]
    K = sv.gram(x, x, 1)
    kc = classical.rbf_gram(x, x, 1.0 / x.shape[1])
    with open(os.path.join(HERE, "c1_eq7.json"), "w") as f:
        json.dump({
            "source": "oracle.statevector.gram (Eq. (7)), oracle.classical (Eqs. (3), (11))",
            "workload": "clusters seed 1, first 24 of 200 samples, d=8, L=1",
            "kq": K.tolist(), "kc": kc.tolist(), "k_w0.5": classical.mix(K, kc, 0.5).tolist(),
        }, f)
    xtr, xte, _ = config_inputs("C3")
    pairs = c3_subset_pairs(xtr.shape[0], xte.shape[0])
    lnk, kcs = [], []
    for rs, i, j in pairs:
        xi = (xtr if rs == 0 else xte)[i]
        xj = xtr[j]
        lnk.append(float(pathsum.ln_kernel_pairs(xi[None], xj[None], 2, [(0, 0)])[0]))
        kcs.append(float(classical.rbf_gram(xi[None], xj[None], 1.0 / 784)[0, 0]))
    kq = [math.exp(v) for v in lnk]
    with open(os.path.join(HERE, "c3_pathsum_200.json"), "w") as f:
        json.dump({
            "source": "oracle.pathsum.ln_kernel_pairs (exact chain), oracle.classical",
            "workload": "images seed 3, 4000 train + 1000 test, d=784, L=2",
            "pairs": pairs, "lnkq": lnk, "kq": kq, "kc": kcs,
            "k_w0.5": [0.5 * a + 0.5 * b for a, b in zip(kq, kcs)],
        }, f)


def s1_replay():
    x, _, _ = config_inputs("S1", n_train=3, n_test=0)
    built = [mps.build_mps(xi, 8, 64, 1e-10, return_discarded=True) for xi in x]
    chi = [list(map(int, b[1])) for b in built]
    discarded = [float(b[2]) for b in built]
    P = mps.pad_batch([b[0] for b in built])
    _, LN = mps.gram(P, P, symmetric=True)
    with open(os.path.join(HERE, "s1_replay_3.json"), "w") as f:
        json.dump({
            "source": "oracle.mps.build_mps (TEBD replay), oracle.mps.gram (FP64 sweep)",
            "workload": "images seed 6, first 3 training samples, d=784, L=8, chi_max=64, "
                        "cutoff 1e-10",
            "chi": chi, "lnkq": LN.tolist(),
            "discarded": discarded,
        }, f)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "s1":
        s1_replay()
    else:
        main()
        s1_replay()
