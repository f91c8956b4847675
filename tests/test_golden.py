"""Stored expected values (tests/golden/) reproduced by the MPS oracle route.

The fixtures come from independent routes (statevector, path-sum), written
by tests/golden/make_golden.py, which calls only the oracle.
"""
import json
import os

import numpy as np

from oracle import checks, classical, mps
from synthdata import config_inputs

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_c1_statevector_fixture():
    g = json.load(open(os.path.join(HERE, "c1_eq7.json")))
    x, _, _ = config_inputs("C1")
    x = x[:24]
    P = mps.pad_batch(mps.build_batch(x, 1, 16))
    K, _ = mps.gram(P, P, symmetric=True)
    assert np.allclose(K, np.array(g["kq"]), rtol=1e-9, atol=1e-13)
    kc = classical.rbf_gram(x, x, 1 / 8)
    assert np.allclose(kc, np.array(g["kc"]), rtol=1e-14, atol=0)


def test_c3_pathsum_fixture_subset():
    g = json.load(open(os.path.join(HERE, "c3_pathsum_200.json")))
    xtr, xte, _ = config_inputs("C3")
    pairs = g["pairs"][:25] + g["pairs"][-15:]
    ln_ref = np.array(g["lnkq"][:25] + g["lnkq"][-15:])
    need = sorted({(rs, i) for rs, i, _ in pairs} | {(0, j) for _, _, j in pairs})
    idx = {k: n for n, k in enumerate(need)}
    X = np.stack([(xtr if rs == 0 else xte)[i] for rs, i in need])
    P = mps.pad_batch(mps.build_batch(X, 2, 64))
    pp = [(idx[(rs, i)], idx[(0, j)]) for rs, i, j in pairs]
    ln = mps.ln_kernel_pairs(P, P, pp)
    ok, err = checks.gate_b(ln, ln_ref, tol=1e-7)
    assert ok, err
