"""MPS simulation of the encoding circuit and the pairwise overlap sweep (oracle).

Site tensors use the index order (left bond, physical, right bond); bond 0
and bond n have dimension 1.

Build (per sample, FP64), a time-evolving-block-decimation replay of the
circuit (the paper contracts the overlap network exactly, Section II-C; the
MPS route reaches the same K_q and makes the work linear in the sample
count). Start from the product state |0...0>, every bond 1. For layer
l = 1..L:

1. apply G_k = RZ(2 x_k) H to the physical index of every site (a unitary on
   that index keeps any canonical form and the orthogonality centre);
2. apply the RZZ chain as two-site steps along the chain, left to right on
   odd layers (k = 0..n-2) and right to left on even layers (k = n-2..0), so
   the orthogonality centre is always one of the two sites merged:
   Theta[(l s), (t r)] = sum_b A_k[l,s,b] A_{k+1}[b,t,r] times the diagonal
   phase exp(-i theta_k/2 sigma_s sigma_t); SVD Theta = U S V^dagger; keep
   the singular values s_j > cutoff * s_0 (at most chi_max, largest first);
   renormalise the kept values to unit norm; then
   left-to-right:  A_k = U (left-canonical),  A_{k+1} = S V^dagger (centre);
   right-to-left:  A_k = U S (centre),        A_{k+1} = V^dagger.

The entanglers of one layer commute, so the sweep direction changes nothing
when no bond is truncated; alternating directions removes the separate
canonicalisation pass a fixed direction would need.

Truncation is per sample, so every sample stays a normalised state and the
Gram matrix of the truncated states is still a Gram matrix (PSD, unit
diagonal).

Sweep (per pair): E_0 = [1]; E_{k+1} = sum_s A_k^{s dagger} E_k B_k^s (a
chi_A x chi_B matrix); after every site E is divided by 2^e with e the
frexp exponent of max(|Re E|, |Im E|) and e is added to an integer
exponent. The overlap <psi_A|psi_B> = E_n * 2^{sum e}; K_q = |.|^2 (Eq. (7)),
ln K_q = 2 (ln|E_n| + sum e * ln 2).
"""
import math

import numpy as np

from .circuit import HADAMARD, entangler_mask, rz, rzz_angles

_SIGMA = np.array([1.0, -1.0])


def build_mps(x, n_layers: int, chi_max: int, cutoff: float = 1e-10,
              entangle=True, return_discarded: bool = False):
    """TEBD build of |psi(x)>. Returns (list of site tensors, bond dims).

    ``entangle``: False, True (open chain) or an entangler block size B >= 2;
    a pair without an entangler is still a two-site step, with no phase (its
    merged tensor is a product across the cut, so one singular value stays).
    With ``return_discarded`` a third value is returned: the sum over all
    truncations of the discarded weight sum_{j >= keep} s_j^2 / sum_j s_j^2.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    A = []
    for _ in range(n):
        t = np.zeros((1, 2, 1), dtype=np.complex128)
        t[0, 0, 0] = 1.0
        A.append(t)
    theta = (rzz_angles(x) * entangler_mask(n, entangle)) if n > 1 else np.zeros(0)
    discarded = 0.0
    for layer in range(n_layers):
        # 1. single-qubit layer
        for k in range(n):
            g = rz(2.0 * x[k]) @ HADAMARD
            A[k] = np.einsum("st,atb->asb", g, A[k])
        if n == 1:
            continue
        # 2. entangler chain, direction alternating with the layer
        left_to_right = (layer % 2 == 0)
        order = range(n - 1) if left_to_right else range(n - 2, -1, -1)
        for k in order:
            chl = A[k].shape[0]
            chr_ = A[k + 1].shape[2]
            th = np.tensordot(A[k], A[k + 1], axes=([2], [0]))  # (l, s, t, r)
            phase = np.exp(-0.5j * theta[k] * np.outer(_SIGMA, _SIGMA))
            th = th * phase[None, :, :, None]
            u, s, vh = np.linalg.svd(th.reshape(chl * 2, 2 * chr_),
                                     full_matrices=False)
            keep = int(np.count_nonzero(s > cutoff * s[0]))
            keep = max(1, min(keep, chi_max))
            discarded += float(np.sum(s[keep:] ** 2) / np.sum(s ** 2))
            u, s, vh = u[:, :keep], s[:keep], vh[:keep]
            s = s / np.linalg.norm(s)
            if left_to_right:
                A[k] = u.reshape(chl, 2, keep)
                A[k + 1] = (s[:, None] * vh).reshape(keep, 2, chr_)
            else:
                A[k] = (u * s[None, :]).reshape(chl, 2, keep)
                A[k + 1] = vh.reshape(keep, 2, chr_)
    chis = [1] + [A[k].shape[2] for k in range(n)]
    if return_discarded:
        return A, chis, discarded
    return A, chis


def build_batch(X, n_layers: int, chi_max: int, cutoff: float = 1e-10,
                entangle=True):
    """Build every row of X; returns a list of MPS (lists of site tensors)."""
    return [build_mps(x, n_layers, chi_max, cutoff, entangle)[0] for x in X]


def pad_batch(mps_list):
    """Stack a batch site by site, zero-padding bonds to the batch maximum.

    Zero padding leaves every overlap unchanged. Returns a list over sites
    of arrays of shape (N, chi_l, 2, chi_r).
    """
    n = len(mps_list[0])
    out = []
    for k in range(n):
        cl = max(m[k].shape[0] for m in mps_list)
        cr = max(m[k].shape[2] for m in mps_list)
        arr = np.zeros((len(mps_list), cl, 2, cr), dtype=np.complex128)
        for i, m in enumerate(mps_list):
            t = m[k]
            arr[i, :t.shape[0], :, :t.shape[2]] = t
        out.append(arr)
    return out


def overlap_pairs(padA, padB, pairs):
    """<psi_A[i]|psi_B[j]> for (i, j) in pairs, as (mantissa, exponent)."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    ia, jb = pairs[:, 0], pairs[:, 1]
    P = pairs.shape[0]
    E = np.ones((P, 1, 1), dtype=np.complex128)
    e2 = np.zeros(P, dtype=np.int64)
    for Ak, Bk in zip(padA, padB):
        a = Ak[ia]
        b = Bk[jb]
        new = np.zeros((P, a.shape[3], b.shape[3]), dtype=np.complex128)
        for s in range(2):
            new += np.conj(a[:, :, s, :]).transpose(0, 2, 1) @ (E @ b[:, :, s, :])
        E = new
        m = np.maximum(np.abs(E.real).reshape(P, -1).max(axis=1),
                       np.abs(E.imag).reshape(P, -1).max(axis=1))
        _, e = np.frexp(np.where(m > 0, m, 1.0))
        E = np.ldexp(E.real, -e[:, None, None]) + 1j * np.ldexp(E.imag, -e[:, None, None])
        e2 += e
    return E[:, 0, 0], e2


def ln_kernel_pairs(padA, padB, pairs):
    """ln K_q per pair (FP64, -inf for an exactly zero overlap)."""
    a, e2 = overlap_pairs(padA, padB, pairs)
    with np.errstate(divide="ignore"):
        return 2.0 * (np.log(np.abs(a)) + e2 * math.log(2.0))


def gram(padA, padB, symmetric: bool = False):
    """Full K_q and ln K_q matrices between two padded batches."""
    NA = padA[0].shape[0]
    NB = padB[0].shape[0]
    ii, jj = np.meshgrid(np.arange(NA), np.arange(NB), indexing="ij")
    pairs = np.stack([ii.ravel(), jj.ravel()], axis=1)
    if symmetric:
        pairs = pairs[pairs[:, 1] >= pairs[:, 0]]
    ln = ln_kernel_pairs(padA, padB, pairs)
    LN = np.full((NA, NB), np.nan)
    LN[pairs[:, 0], pairs[:, 1]] = ln
    if symmetric:
        LN[pairs[:, 1], pairs[:, 0]] = ln
    return np.exp(LN), LN


def to_state(mps) -> np.ndarray:
    """Contract an MPS into a dense vector (small n only)."""
    v = mps[0]
    for t in mps[1:]:
        v = np.tensordot(v, t, axes=([-1], [0]))
    return v.reshape(-1)
