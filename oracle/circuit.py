"""Gates and angles of the encoding circuit (oracle side).

The paper's feature map (Eq. (6); Section II-C, Fig. 1(B)) interleaves
Hadamards and data-dependent single-qubit rotations with locally restricted
entangling layers. The benchmark instance used throughout is, per layer:

    H on every qubit  ->  RZ(2 x_k) on qubit k  ->  RZZ(theta_k) on (k, k+1),
    k = 0 .. n-2 (open chain), theta_k = 2 (pi - x_k)(pi - x_{k+1}),

repeated L times with the same x. Conventions: RZ(phi) = exp(-i phi Z / 2),
RZZ(theta) = exp(-i theta Z(x)Z / 2), basis |0> = (1, 0).

Block-structured entanglers (the block product state circuits the paper
names): the qubits are cut into blocks of B consecutive qubits and the RZZ
chain keeps only the pairs (k, k+1) inside one block, i.e. drops the pairs
with (k + 1) divisible by B. The argument ``entangle`` of the oracle
functions takes False / 0 (no entanglers), True / 1 (the open chain over all
qubits) or a block size B >= 2.
"""
import math

import numpy as np

HADAMARD = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / math.sqrt(2.0)


def rz(phi: float) -> np.ndarray:
    """RZ(phi) = diag(exp(-i phi/2), exp(+i phi/2))."""
    return np.diag([np.exp(-0.5j * phi), np.exp(0.5j * phi)])


def rzz(theta: float) -> np.ndarray:
    """RZZ(theta) on basis |00>,|01>,|10>,|11>: diag(e^-, e^+, e^+, e^-)."""
    m = np.exp(-0.5j * theta)
    p = np.exp(0.5j * theta)
    return np.diag([m, p, p, m])


def rz_angles(x: np.ndarray) -> np.ndarray:
    """Single-qubit rotation angles phi_k = 2 x_k."""
    return 2.0 * np.asarray(x, dtype=np.float64)


def rzz_angles(x: np.ndarray) -> np.ndarray:
    """Entangler angles theta_k = 2 (pi - x_k)(pi - x_{k+1}), k = 0..n-2."""
    x = np.asarray(x, dtype=np.float64)
    return 2.0 * (math.pi - x[:-1]) * (math.pi - x[1:])


def entangler_mask(n: int, entangle=True) -> np.ndarray:
    """Boolean array of length n-1: whether RZZ acts on the pair (k, k+1)."""
    m = max(n - 1, 0)
    if entangle is False or entangle == 0:
        return np.zeros(m, dtype=bool)
    if entangle is True or entangle == 1:
        return np.ones(m, dtype=bool)
    B = int(entangle)
    if B < 2:
        raise ValueError("entangle must be False/0, True/1 or a block size >= 2")
    return np.array([(k + 1) % B != 0 for k in range(m)], dtype=bool)
