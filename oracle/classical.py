"""Classical RBF kernel (Eq. (3)), the quantum-classical mix (Eq. (11)) and
the SVM decision function on kernel rows (Eqs. (4), (5)).

* K_c(x, y) = exp(-gamma ||x - y||^2), evaluated by direct differences.
  The benchmark workloads use gamma = 1/d.
* K_{q-c} = w K_q + (1 - w) K_c with w in [0, 1] (the paper's alpha; named
  w here because alpha_i are the SVM multipliers of Eqs. (1)-(2)).
* f(x) = sum_i alpha_i y_i K(x_i, x) + b, the label being sign(f); coef_i =
  alpha_i y_i (zero off the support vectors).
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


def svm_decision(k_rows, coef, b: float) -> np.ndarray:
    """f[r] = sum_i coef[i] K[r][i] + b, term by term in FP64."""
    K = np.asarray(k_rows, dtype=np.float64)
    c = np.asarray(coef, dtype=np.float64)
    out = np.empty(K.shape[0])
    for r in range(K.shape[0]):
        acc = 0.0
        for i in range(K.shape[1]):
            acc += c[i] * K[r, i]
        out[r] = acc + b
    return out
