"""Exact path-sum evaluation of <psi(x)|psi(y)> for any qubit count (oracle).

Independent of the MPS route; used to pin it at full size (hundreds of
qubits). Every gate of the encoding circuit except H is diagonal in the
computational basis, so expanding each Hadamard layer as
H|z> = 2^{-1/2} sum_{z'} (-1)^{z z'} |z'> writes an amplitude as a sum over
basis histories z^(1), ..., z^(L) (z^(0) = 0):

    psi_x(z^(L)) = 2^{-nL/2} sum_{z^(1..L-1)} prod_l (-1)^{z^(l-1).z^(l)}
                   exp(-i Phi_x(z^(l))),
    Phi_x(z) = sum_k x_k s_k + sum_k (theta_k(x)/2) s_k s_{k+1},
    s_k = (-1)^{z_k}.

The overlap <psi(x)|psi(y)> sums conj(psi_x) psi_y over a history u for x, a
history v for y, and the shared last layer z = u^(L) = v^(L). All factors
are products over sites and nearest-neighbour bonds, so with the per-site
state c_k = (u_k^(1..L-1), v_k^(1..L-1), z_k) (2^(2L-1) values) the sum is a
transfer chain:

    weight w_k(c)    = 2^{-L} (-1)^{sum_l u^(l-1)u^(l) + v^(l-1)v^(l)}
                        exp(i x_k sum_l s(u^(l)) - i y_k sum_l s(v^(l))),
    coupling J_k(c,c') = exp(i theta_k(x)/2 sum_l s(u^(l))s(u'^(l))
                             - i theta_k(y)/2 sum_l s(v^(l))s(v'^(l))),

    a = sum_{c_0..c_{n-1}} prod_k w_k(c_k) prod_k J_k(c_k, c_{k+1}).

The chain vector is rescaled by an exact power of two at every site, so the
result is returned as (mantissa, base-2 exponent) and ln K is exact in range.
"""
import itertools
import math

import numpy as np

from .circuit import entangler_mask, rzz_angles


def _site_tables(n_layers: int):
    L = n_layers
    nb = 2 * L - 1
    states = list(itertools.product((0, 1), repeat=nb))
    S = len(states)
    su = np.zeros(S)          # sum_l s(u^(l)), l = 1..L
    sv = np.zeros(S)
    sign = np.zeros(S)
    lines_u = np.zeros((S, L))
    lines_v = np.zeros((S, L))
    for idx, c in enumerate(states):
        u = list(c[:L - 1]) + [c[-1]]
        v = list(c[L - 1:2 * L - 2]) + [c[-1]]
        su_ = [1 - 2 * b for b in u]
        sv_ = [1 - 2 * b for b in v]
        su[idx] = sum(su_)
        sv[idx] = sum(sv_)
        par = 0
        prev_u, prev_v = 0, 0
        for l in range(L):
            par += prev_u * u[l] + prev_v * v[l]
            prev_u, prev_v = u[l], v[l]
        sign[idx] = -1.0 if (par & 1) else 1.0
        lines_u[idx] = su_
        lines_v[idx] = sv_
    pu = lines_u @ lines_u.T      # sum_l s(u^(l)) s(u'^(l))
    pv = lines_v @ lines_v.T
    return su, sv, sign, pu, pv


def overlap_pairs(X, Y, n_layers: int, pairs, entangle=True):
    """<psi(X[i])|psi(Y[j])> for (i, j) in pairs (``entangle``: False, True
    for the open chain, or an entangler block size B >= 2).

    Returns (mant, exp2): complex mantissas and integer exponents with
    a = mant * 2**exp2.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    L = n_layers
    n = X.shape[1]
    su, sv, sign, pu, pv = _site_tables(L)
    xi = X[pairs[:, 0]]
    yj = Y[pairs[:, 1]]
    P = pairs.shape[0]
    if n > 1:
        on = entangler_mask(n, entangle)
        tx = np.stack([rzz_angles(r) for r in xi]) * on
        ty = np.stack([rzz_angles(r) for r in yj]) * on
    else:
        tx = np.zeros((P, max(n - 1, 0)))
        ty = np.zeros((P, max(n - 1, 0)))
    scale = 2.0 ** (-L)

    def weight(k):
        ph = xi[:, k:k + 1] * su[None, :] - yj[:, k:k + 1] * sv[None, :]
        return scale * sign[None, :] * np.exp(1j * ph)

    v = weight(0)
    e2 = np.zeros(P, dtype=np.int64)
    for k in range(n - 1):
        J = np.exp(1j * (0.5 * tx[:, k, None, None] * pu[None]
                         - 0.5 * ty[:, k, None, None] * pv[None]))
        v = np.einsum("pc,pcd->pd", v, J) * weight(k + 1)
        m = np.maximum(np.abs(v.real).max(axis=1), np.abs(v.imag).max(axis=1))
        _, e = np.frexp(np.where(m > 0, m, 1.0))
        v = np.ldexp(v.real, -e[:, None]) + 1j * np.ldexp(v.imag, -e[:, None])
        e2 += e
    a = v.sum(axis=1)
    return a, e2


def ln_kernel_pairs(X, Y, n_layers: int, pairs, entangle=True):
    """ln K_q = 2 ln|a| for each pair (-inf where a == 0)."""
    a, e2 = overlap_pairs(X, Y, n_layers, pairs, entangle)
    with np.errstate(divide="ignore"):
        return 2.0 * (np.log(np.abs(a)) + e2 * math.log(2.0))
