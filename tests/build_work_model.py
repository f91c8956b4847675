"""Work model of the device TEBD build in the truncating regime.

The large-bond build factors every merged two-site matrix (R = 2 chi_l rows,
C = 2 chi_r columns) by a one-sided Jacobi method: column pairs meet in the
round-robin order of the workgroup kernel (C - 1 rounds per sweep), a pair
rotates when |g|^2 > tol^2 a b (g = x_p^H x_q, a and b the squared column
norms, tol 1e-14) and both norms exceed 1e-30 of the matrix's squared
Frobenius norm, and the sweeps stop after the first sweep without a
rotation. The number of sweeps is data-dependent and the device does not
report it, so this model replays the oracle's build of one sample
(Section II-C, Eq. 6; LAPACK's SVD continues the build) and runs the same
rule on the merged matrices of every `every`-th step, then tallies the
arithmetic of each step:

  forming Theta         8 R C chi_m      (complex MACs, 8 real FLOP each)
  Jacobi, per sweep     C (C - 1) / 2 column pairs x 16 R (three dot products)
  Jacobi, per rotation  14 R             (phase, then the 2 x 2 rotation)
  right factor U^H Theta   8 keep R C

The merged matrices differ from the device's by the gauge of earlier steps
(phases of singular vectors), which leaves column norms and |g| unchanged
and the sweep counts close to, not equal to, the device's.

Test infrastructure: run as `python -m tests.build_work_model [every]
[build_seconds samples]` from the repository root for the FLOP tally, or
with `--orderings` for the sweep counts of alternative Jacobi set-ups on
the last layer's full-bond matrices.
"""
import math
import sys

import numpy as np

from oracle.circuit import HADAMARD, entangler_mask, rz, rzz_angles

_SIGMA = np.array([1.0, -1.0])


def round_robin_rounds(C):
    """Column pairs of each round: start (p, C-1-p); after a round slot 0
    keeps its first column, slot 1 takes slot 0's second, slot p >= 2 takes
    slot p-1's first, slot p < P-1 takes slot p+1's second, the last slot
    its own first."""
    P = C // 2
    cur = [(p, C - 1 - p) for p in range(P)]
    rounds = []
    for _ in range(C - 1):
        rounds.append((np.array([a for a, _ in cur]), np.array([b for _, b in cur])))
        if P >= 2:
            nxt = []
            for p in range(P):
                first = cur[0][0] if p == 0 else (cur[0][1] if p == 1 else cur[p - 1][0])
                second = cur[p][0] if p == P - 1 else cur[p + 1][1]
                nxt.append((first, second))
            cur = nxt
    return rounds


def jacobi_model(X, tol=1e-14, max_sweeps=1000, floor=1e-30):
    """One-sided Jacobi under the device's rule (tolerance 1e-14, squared
    column-norm floor 1e-30 of the matrix's; both can be varied to study
    the sweep count). Returns (singular values in decreasing order, sweeps
    including the final one without a rotation, rotations applied)."""
    X = np.array(X, dtype=np.complex128, copy=True)
    R, C = X.shape
    if C % 2:
        X = np.concatenate([X, np.zeros((R, 1), X.dtype)], axis=1)
        C += 1
    floor2 = floor * float(np.sum(np.abs(X) ** 2))
    rounds = round_robin_rounds(C)
    rotations = 0
    sweeps = max_sweeps
    for sweep in range(max_sweeps):
        rotated = False
        for ip, iq in rounds:
            xp, xq = X[:, ip], X[:, iq]
            a = np.sum(np.abs(xp) ** 2, axis=0)
            b = np.sum(np.abs(xq) ** 2, axis=0)
            g = np.sum(np.conj(xp) * xq, axis=0)
            g2 = np.abs(g) ** 2
            do = (a > floor2) & (b > floor2) & (g2 > tol * tol * a * b)
            if not do.any():
                continue
            rotated = True
            rotations += int(do.sum())
            ig = 1.0 / np.sqrt(np.where(do, g2, 1.0))
            zeta = 0.5 * (b - a) * ig
            t = np.where(zeta >= 0, 1.0, -1.0) / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta))
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            b0 = (np.conj(g) * ig) * xq
            X[:, ip] = np.where(do, c * xp - s * b0, xp)
            X[:, iq] = np.where(do, s * xp + c * b0, xq)
        if not rotated:
            sweeps = sweep + 1
            break
    sv = np.sort(np.sqrt(np.sum(np.abs(X) ** 2, axis=0)))[::-1]
    return sv, sweeps, rotations


def preconditioned_jacobi(X, twice=False):
    """The same rule on R^H after a Householder QR with column pivoting of X
    (X P = Q R; R^H has the singular values of X, and for graded matrices
    its columns are close to orthogonal already), optionally after a second
    QR without pivoting (R^H = Q2 R2, Jacobi on R2^H). Returns what
    jacobi_model returns."""
    import scipy.linalg as sl
    _, Rm, _ = sl.qr(np.asarray(X, dtype=np.complex128), pivoting=True, mode="economic")
    Y = Rm.conj().T
    if twice:
        _, R2 = np.linalg.qr(Y)
        Y = R2.conj().T
    return jacobi_model(Y)


def merged_matrices(x, n_layers, chi_max, layer, every, cutoff=1e-10, full_bond_only=True):
    """The merged two-site matrices of one layer of the oracle's build of one
    sample (every `every`-th step; by default only steps whose bonds are both
    at the cap)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    A = [np.array([[[1.0], [0.0]]], dtype=np.complex128) for _ in range(n)]
    theta = rzz_angles(x) * entangler_mask(n, True)
    mats = []
    for lay in range(layer + 1):
        for k in range(n):
            A[k] = np.einsum("st,atb->asb", rz(2.0 * x[k]) @ HADAMARD, A[k])
        l2r = lay % 2 == 0
        order = range(n - 1) if l2r else range(n - 2, -1, -1)
        for idx, k in enumerate(order):
            chl, chr_ = A[k].shape[0], A[k + 1].shape[2]
            th = np.tensordot(A[k], A[k + 1], axes=([2], [0]))
            th = th * np.exp(-0.5j * theta[k] * np.outer(_SIGMA, _SIGMA))[None, :, :, None]
            M = th.reshape(chl * 2, 2 * chr_)
            if lay == layer and idx % every == every // 2 and (
                    not full_bond_only or (chl == chi_max and chr_ == chi_max)):
                mats.append(M.copy())
            u, s, vh = np.linalg.svd(M, full_matrices=False)
            keep = max(1, min(int(np.count_nonzero(s > cutoff * s[0])), chi_max))
            u, s, vh = u[:, :keep], s[:keep], vh[:keep]
            s = s / np.linalg.norm(s)
            if l2r:
                A[k] = u.reshape(chl, 2, keep)
                A[k + 1] = (s[:, None] * vh).reshape(keep, 2, chr_)
            else:
                A[k] = (u * s[None, :]).reshape(chl, 2, keep)
                A[k + 1] = vh.reshape(keep, 2, chr_)
    return mats


def step_flop(R, C, chi_m, keep, sweeps, rotations):
    Ce = C + (C % 2)
    return (8.0 * R * C * chi_m + sweeps * (Ce * (Ce - 1) / 2) * 16.0 * R
            + rotations * 14.0 * R + 8.0 * keep * R * C)


def work_of_sample(x, n_layers, chi_max, cutoff=1e-10, every=8):
    """Per layer: steps, sampled steps, mean sweeps of the sampled steps,
    and the layer's FLOP (the Jacobi part scaled from the sampled steps by
    R C^2)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    A = [np.array([[[1.0], [0.0]]], dtype=np.complex128) for _ in range(n)]
    theta = rzz_angles(x) * entangler_mask(n, True)
    out = []
    for layer in range(n_layers):
        for k in range(n):
            A[k] = np.einsum("st,atb->asb", rz(2.0 * x[k]) @ HADAMARD, A[k])
        l2r = layer % 2 == 0
        order = range(n - 1) if l2r else range(n - 2, -1, -1)
        fixed = jac_s = w_s = w_all = 0.0
        sweeps = []
        for idx, k in enumerate(order):
            chl, chm, chr_ = A[k].shape[0], A[k].shape[2], A[k + 1].shape[2]
            th = np.tensordot(A[k], A[k + 1], axes=([2], [0]))
            th = th * np.exp(-0.5j * theta[k] * np.outer(_SIGMA, _SIGMA))[None, :, :, None]
            M = th.reshape(chl * 2, 2 * chr_)
            u, s, vh = np.linalg.svd(M, full_matrices=False)
            keep = max(1, min(int(np.count_nonzero(s > cutoff * s[0])), chi_max))
            R, C = 2 * chl, 2 * chr_
            fixed += step_flop(R, C, chm, keep, 0, 0)
            w_all += R * C * C
            if idx % every == 0:
                _, S, rot = jacobi_model(M)
                jac_s += step_flop(R, C, 0, 0, S, rot)
                w_s += R * C * C
                sweeps.append(S)
            u, s, vh = u[:, :keep], s[:keep], vh[:keep]
            s = s / np.linalg.norm(s)
            if l2r:
                A[k] = u.reshape(chl, 2, keep)
                A[k + 1] = (s[:, None] * vh).reshape(keep, 2, chr_)
            else:
                A[k] = (u * s[None, :]).reshape(chl, 2, keep)
                A[k + 1] = vh.reshape(keep, 2, chr_)
        out.append({"layer": layer + 1, "steps": n - 1, "sampled": len(sweeps),
                    "mean_sweeps": float(np.mean(sweeps)), "max_sweeps": int(max(sweeps)),
                    "flop_fixed": fixed, "flop_jacobi": jac_s / w_s * w_all})
    return out


def compare_orderings(x, every=30):
    """Sweeps of the device rule on the last layer's full-bond merged
    matrices, against a looser tolerance, a column-norm floor at the
    truncation cutoff, and QR-preconditioned Jacobi (once and twice)."""
    mats = merged_matrices(x, 8, 64, 7, every)
    rows = []
    for M in mats:
        ref = np.linalg.svd(M, compute_uv=False)
        out = {}
        for name, (sv, S, _) in (("device rule", jacobi_model(M)),
                                 ("tolerance 1e-8", jacobi_model(M, tol=1e-8)),
                                 ("floor at the cutoff", jacobi_model(M, floor=1e-20)),
                                 ("QR with pivoting, then Jacobi on R^H", preconditioned_jacobi(M)),
                                 ("two QRs, then Jacobi", preconditioned_jacobi(M, True))):
            k = min(64, len(ref))
            out[name] = (S, float(np.max(np.abs(sv[:k] - ref[:k])) / ref[0]))
        rows.append(out)
    return rows


if __name__ == "__main__":
    from synthdata import config_inputs

    if len(sys.argv) > 1 and sys.argv[1] == "--orderings":
        x, _, _ = config_inputs("S1", n_train=1, n_test=0)
        rows = compare_orderings(x[0])
        print(f"{len(rows)} merged 128 x 128 matrices of layer 8")
        for name in rows[0]:
            S = [r[name][0] for r in rows]
            e = max(r[name][1] for r in rows)
            print(f"{name}: sweeps {min(S)}..{max(S)} (mean {np.mean(S):.1f}); "
                  f"kept singular values within {e:.1e} s_0 of LAPACK's")
        sys.exit(0)
    every = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    x, _, _ = config_inputs("S1", n_train=1, n_test=0)
    rows = work_of_sample(x[0], 8, 64, 1e-10, every)
    tot = 0.0
    for r in rows:
        t = r["flop_fixed"] + r["flop_jacobi"]
        tot += t
        print(f"layer {r['layer']}: {r['sampled']} of {r['steps']} steps sampled, sweeps mean "
              f"{r['mean_sweeps']:.1f} max {r['max_sweeps']}; {t:.3g} FLOP "
              f"({100 * r['flop_jacobi'] / t:.0f} % Jacobi)", flush=True)
    print(f"per sample: {tot:.4g} FLOP")
    if len(sys.argv) > 3:
        secs, samples = float(sys.argv[2]), int(sys.argv[3])
        rate = tot * samples / secs / 1e12
        print(f"{samples} samples in {secs} s: {rate:.2f} TFLOP/s, {100 * rate / 78.6:.1f} % of 78.6")
