"""Gates and angles of the encoding circuit (oracle side).

The paper's feature map (Eq. (6); Section II-C, Fig. 1(B)) interleaves
Hadamards and data-dependent single-qubit rotations with locally restricted
entangling layers. The benchmark instance used throughout is, per layer:

    H on every qubit  ->  RZ(2 x_k) on qubit k  ->  RZZ(theta_k) on (k, k+1),
    k = 0 .. n-2 (open chain), theta_k = 2 (pi - x_k)(pi - x_{k+1}),

repeated L times with the same x. Conventions: RZ(phi) = exp(-i phi Z / 2),
RZZ(theta) = exp(-i theta Z(x)Z / 2), basis |0> = (1, 0).
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
