"""Classical RBF kernel (Eq. (3)) and the quantum-classical mix (Eq. (11)).

* K_c(x, y) = exp(-gamma ||x - y||^2), evaluated by direct differences.
  The benchmark workloads use gamma = 1/d.
* K_{q-c} = w K_q + (1 - w) K_c with w in [0, 1] (the paper's alpha; named
  w here because alpha_i are the SVM multipliers of Eqs. (1)-(2)).
"""
import numpy as np


def rbf_gram(X, Y, gamma: float) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty((X.shape[0], Y.shape[0]))
    for i in range(X.shape[0]):
        diff = X[i][None, :] - Y
        out[i] = np.exp(-gamma * np.sum(diff * diff, axis=1))
    return out


def mix(kq, kc, w: float) -> np.ndarray:
    return w * np.asarray(kq) + (1.0 - w) * np.asarray(kc)
