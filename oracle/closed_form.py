"""Entangler-free closed forms of the quantum kernel (oracle).

With every RZZ angle set to zero the circuit of Eq. (6) is a product of
single-qubit circuits (RZ(2 x_k) H)^L |0>, so Eq. (7) factorises into a
product of per-qubit overlaps. Worked by hand:

* L = 1: (RZ(2x) H)|0> = (e^{-ix}|0> + e^{ix}|1>)/sqrt(2), and the per-qubit
  overlap is cos(x - y), so K_q = prod_k cos^2(x_k - y_k).
* L = 2: (RZ(2x) H)^2 |0> = (e^{-ix} cos x, -i e^{ix} sin x), and the
  per-qubit overlap is cos x cos y e^{i(x-y)} + sin x sin y e^{-i(x-y)}.
* any L: multiply the 2x2 matrices out per qubit (``kernel_product``).
"""
import numpy as np

from .circuit import HADAMARD, rz


def kernel_L1(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.prod(np.cos(x - y) ** 2))


def kernel_L2(x, y) -> float:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    ov = (np.cos(x) * np.cos(y) * np.exp(1j * (x - y))
          + np.sin(x) * np.sin(y) * np.exp(-1j * (x - y)))
    return float(np.prod(np.abs(ov) ** 2))


def single_qubit_state(xk: float, n_layers: int) -> np.ndarray:
    v = np.array([1.0, 0.0], dtype=np.complex128)
    g = rz(2.0 * xk) @ HADAMARD
    for _ in range(n_layers):
        v = g @ v
    return v


def kernel_product(x, y, n_layers: int) -> float:
    """prod_k |<phi_L(x_k)|phi_L(y_k)>|^2 for any L (entanglers off)."""
    out = 1.0
    for xk, yk in zip(x, y):
        out *= abs(np.vdot(single_qubit_state(xk, n_layers),
                           single_qubit_state(yk, n_layers))) ** 2
    return float(out)
