"""Brute-force statevector evaluation of the quantum kernel (oracle).

Definition of record for small qubit counts (n <= ~16):

* ``state``: |psi(x)> = U(x)|0>^{(x)n}, Eq. (6), built gate by gate.
* ``kernel_overlap``: K_q = |<psi(x)|psi(y)>|^2, Eq. (7).
* ``amplitude_compute_uncompute``: a = <0| U^dagger(y) U(x) |0>, Eqs. (8)-(9),
  by running the gate list of U(x) and then the inverted, reversed gate list
  of U(y); K_q = |a|^2 is Eq. (10).
"""
import numpy as np

from .circuit import HADAMARD, entangler_mask, rz, rzz, rzz_angles


def gate_list(x, n_layers: int, entangle=True):
    """Ordered gates of U(x): list of (qubits, unitary). ``entangle``: False
    (none), True (open chain) or an entangler block size B >= 2 (the chain's
    pairs inside blocks of B qubits only)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    theta = rzz_angles(x) if n > 1 else np.zeros(0)
    on = entangler_mask(n, entangle)
    gates = []
    for _ in range(n_layers):
        for k in range(n):
            gates.append(((k,), HADAMARD))
        for k in range(n):
            gates.append(((k,), rz(2.0 * x[k])))
        for k in range(n - 1):
            if on[k]:
                gates.append(((k, k + 1), rzz(theta[k])))
    return gates


def _apply(psi, qubits, g):
    if len(qubits) == 1:
        (k,) = qubits
        psi = np.tensordot(g, psi, axes=([1], [k]))
        return np.moveaxis(psi, 0, k)
    k, k1 = qubits
    g4 = g.reshape(2, 2, 2, 2)
    psi = np.tensordot(g4, psi, axes=([2, 3], [k, k1]))
    return np.moveaxis(psi, [0, 1], [k, k1])


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def state(x, n_layers: int, entangle=True) -> np.ndarray:
    """|psi(x)> as an n-axis tensor (axis k = qubit k)."""
    n = len(x)
    psi = zero_state(n)
    for q, g in gate_list(x, n_layers, entangle):
        psi = _apply(psi, q, g)
    return psi


def kernel_overlap(x, y, n_layers: int, entangle=True) -> float:
    """Eq. (7): |<psi(x)|psi(y)>|^2."""
    a = np.vdot(state(x, n_layers, entangle), state(y, n_layers, entangle))
    return float(abs(a) ** 2)


def amplitude_compute_uncompute(x, y, n_layers: int, entangle=True):
    """Eqs. (8)-(9): <0| U^dagger(y) U(x) |0>, gate by gate."""
    n = len(x)
    psi = zero_state(n)
    for q, g in gate_list(x, n_layers, entangle):
        psi = _apply(psi, q, g)
    for q, g in reversed(gate_list(y, n_layers, entangle)):
        psi = _apply(psi, q, g.conj().T)
    return complex(psi[(0,) * n])


def gram(X, Y, n_layers: int, entangle=True) -> np.ndarray:
    """Eq. (7) for all pairs of rows of X and Y."""
    sx = [state(x, n_layers, entangle).ravel() for x in X]
    sy = [state(y, n_layers, entangle).ravel() for y in Y]
    A = np.array(sx)
    B = np.array(sy)
    return np.abs(A.conj() @ B.T) ** 2
