"""Helpers shared by the GPU parity tests (oracle side and data marshalling)."""
import numpy as np

from oracle import mps


def oracle_import_layout(mps_list, T):
    """Pack oracle MPS (lists of (l, s, r) tensors) into the import layout
    [site][sample][s][a][b] (complex128, padded to T) plus the bond table."""
    n = len(mps_list)
    nq = len(mps_list[0])
    ten = np.zeros((nq, n, 2, T, T), dtype=np.complex128)
    chi = np.ones((n, nq + 1), dtype=np.int32)
    for i, m in enumerate(mps_list):
        for k, t in enumerate(m):
            l, _, r = t.shape
            ten[k, i, :, :l, :r] = t.transpose(1, 0, 2)
            chi[i, k + 1] = r
    return chi, ten


def oracle_gram(X, L, chi_max, symmetric=False, Y=None):
    P = mps.pad_batch(mps.build_batch(X, L, chi_max))
    Q = P if Y is None else mps.pad_batch(mps.build_batch(Y, L, chi_max))
    return mps.gram(P, Q, symmetric=symmetric and Y is None)


def oracle_chis(X, L, chi_max):
    return np.array([mps.build_mps(x, L, chi_max)[1] for x in X], dtype=np.int32)


def import_layout_to_oracle(chi, ten):
    """Inverse of oracle_import_layout: per sample, the list of (l, s, r)
    site tensors of its own bond dimensions."""
    nq, n = ten.shape[0], ten.shape[1]
    return [[np.ascontiguousarray(ten[k, i, :, :chi[i, k], :chi[i, k + 1]].transpose(1, 0, 2))
             for k in range(nq)] for i in range(n)]
