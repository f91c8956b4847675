"""Host emulation of the reduced-precision sweep's log-error tail.

The transfer sweep of Eqs. (9)-(10), E <- sum_s A^s^H E B^s over the sites,
run with complex64 arithmetic (single-precision products and sums) and an
exact power-of-two rescale of E every 8 sites, against the same sweep in
complex128, on all pairs of a subset of the 784-qubit image workload's
training samples (MPS from the oracle's build). It measures how far
single-precision arithmetic alone moves ln K_q, independent of any device
kernel's operation order, and records for each pair the largest drop of
the max |E| exponent over an 8-site block (a candidate detector of the
pairs that fall outside the log gate).

With `--operands-only` the sweep instead runs in complex128 on site tensors
rounded to complex64: the share of the error that the single-precision
operands alone cause, with exact-enough arithmetic.

Test infrastructure: `python -m tests.fp32_tail_model [n_samples]
[--operands-only]` from the repository root (about 30 minutes for 1200
samples on 8 host cores).
"""
import math
import sys

import numpy as np

from oracle import mps


def sweep(pad, ia, jb, dtype, every=8):
    """ln K_q of the pairs (ia[p], jb[p]) of one padded batch, the sweep run
    in `dtype`, with the largest per-block exponent drop of each pair."""
    P = len(ia)
    E = np.ones((P, 1, 1), dtype=dtype)
    e2 = np.zeros(P, dtype=np.int64)
    drops = np.zeros(P)
    for k, Ak in enumerate(pad):
        a = Ak[ia].astype(dtype)
        b = Ak[jb].astype(dtype)
        new = np.zeros((P, a.shape[3], b.shape[3]), dtype=dtype)
        for s in range(2):
            new += np.conj(a[:, :, s, :]).transpose(0, 2, 1) @ (E @ b[:, :, s, :])
        E = new
        if (k + 1) % every == 0 or k == len(pad) - 1:
            m = np.maximum(np.abs(E.real).reshape(P, -1).max(axis=1),
                           np.abs(E.imag).reshape(P, -1).max(axis=1)).astype(np.float64)
            _, e = np.frexp(np.where(m > 0, m, 1.0))
            E = (np.ldexp(E.real.astype(np.float64), -e[:, None, None])
                 + 1j * np.ldexp(E.imag.astype(np.float64), -e[:, None, None])).astype(dtype)
            drops = np.maximum(drops, -e.astype(np.float64))
            e2 += e
    with np.errstate(divide="ignore"):
        ln = 2.0 * (np.log(np.abs(E[:, 0, 0].astype(np.complex128))) + e2 * math.log(2.0))
    return ln, drops


def _build(x):
    return mps.build_mps(x, 2, 64, 1e-10)[0]


if __name__ == "__main__":
    from multiprocessing import Pool

    from synthdata import config_inputs

    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    operands_only = "--operands-only" in sys.argv
    N = int(args[0]) if args else 1200
    x, _, _ = config_inputs("C3", n_train=N, n_test=0)
    with Pool(8) as pool:
        built = pool.map(_build, list(x), chunksize=8)
    pad = mps.pad_batch(built)
    if operands_only:
        pad_r = [a.astype(np.complex64).astype(np.complex128) for a in pad]
    ia, jb = np.triu_indices(N, 1)
    lab = np.arange(N) % 10
    err, drop, lns = [], [], []
    for c0 in range(0, len(ia), 100000):
        sl = slice(c0, c0 + 100000)
        l64, _ = sweep(pad, ia[sl], jb[sl], np.complex128)
        if operands_only:
            l32, d32 = sweep(pad_r, ia[sl], jb[sl], np.complex128)
        else:
            l32, d32 = sweep(pad, ia[sl], jb[sl], np.complex64)
        err.append(np.abs(l32 - l64))
        drop.append(d32)
        lns.append(l64)
        print(f"{min(c0 + 100000, len(ia))} of {len(ia)} pairs", flush=True)
    err, drop, lns = np.concatenate(err), np.concatenate(drop), np.concatenate(lns)
    same = lab[ia] == lab[jb]
    print(f"{len(err)} off-diagonal pairs: max |d ln K_q| {err.max():.3g}, "
          f"{(err > 1e-3).sum()} above 1e-3, {(err > 1e-4).sum()} above 1e-4; "
          f"same-class max {err[same].max():.3g}, cross-class max {err[~same].max():.3g}")
    tail = err > 1e-3
    print(f"largest 8-site exponent drop: median {np.median(drop):.0f}, max {drop.max():.0f}; "
          f"of the pairs above 1e-3: {np.sort(drop[tail]).astype(int).tolist()}")
    if tail.any():
        print(f"ln K_q of the pairs above 1e-3: {lns[tail].min():.1f} to "
              f"{lns[tail].max():.1f} (all pairs: {lns.min():.1f} to {lns.max():.1f})")
