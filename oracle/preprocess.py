"""Pre-processing of the raw features (Section II-A), oracle side.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper standardises every raw feature to zero mean and unit variance,
applies principal component analysis and keeps the n leading components
(n = the qubit count), and finally min-max scales each kept component to
[0, 1]. Written out, with the statistics fitted on the training rows X
(N x D):

1. z-score: mu_c = mean of column c, sigma_c = sqrt(mean of (x - mu_c)^2)
   (population variance); z = (x - mu_c) / sigma_c, and z = 0 for a
   constant column (sigma_c = 0).
2. PCA: C = Z^T Z / (N - 1) (the sample covariance of the standardised
   training rows); its eigenvectors by decreasing eigenvalue; the n leading
   ones are the components. An eigenvector is defined up to sign: each
   component is taken with its entry of largest magnitude positive (the
   first such entry on ties). The projection is y = z . w_j.
3. min-max: per component, the training rows' minimum m_j and maximum M_j;
   u = (y - m_j) / (M_j - m_j) (0 when M_j = m_j). Training rows land in
   [0, 1]; other rows use the training statistics and may fall outside.
4. The encoding angles are u times a scale (1 in the paper's [0, 1]
   convention; pi for the [0, pi] convention of the benchmark workloads).

Library routines used as steps: numpy means, a matrix product and the
symmetric eigensolver (LAPACK through numpy.linalg.eigh).
"""
import numpy as np


class Fit:
    """Statistics fitted on the training rows."""

    def __init__(self, mu, sigma, components, eigvals, ymin, ymax):
        self.mu = mu
        self.sigma = sigma
        self.components = components  # n x D, one component per row
        self.eigvals = eigvals          # all D eigenvalues, decreasing
        self.ymin = ymin
        self.ymax = ymax


def zscore(X, mu, sigma):
    X = np.asarray(X, dtype=np.float64)
    Z = np.zeros_like(X)
    nz = sigma > 0.0
    Z[:, nz] = (X[:, nz] - mu[nz]) / sigma[nz]
    return Z


def fix_signs(V):
    """Each row of V with its entry of largest magnitude positive."""
    V = np.array(V, dtype=np.float64, copy=True)
    for j in range(V.shape[0]):
        i = int(np.argmax(np.abs(V[j])))  # first maximum on ties
        if V[j, i] < 0.0:
            V[j] = -V[j]
    return V


def fit(X, n_components: int) -> Fit:
    X = np.asarray(X, dtype=np.float64)
    N, D = X.shape
    if not 1 <= n_components <= D:
        raise ValueError("n_components must be in [1, D]")
    mu = X.mean(axis=0)
    sigma = np.sqrt(((X - mu) ** 2).mean(axis=0))
    Z = zscore(X, mu, sigma)
    C = (Z.T @ Z) / (N - 1)
    lam, vecs = np.linalg.eigh(C)           # ascending
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    W = fix_signs(vecs[:, order[:n_components]].T)
    Y = Z @ W.T
    return Fit(mu, sigma, W, lam, Y.min(axis=0), Y.max(axis=0))


def transform(f: Fit, X, scale: float = 1.0):
    """z-score with the fitted statistics, project, min-max, times scale."""
    Y = zscore(X, f.mu, f.sigma) @ f.components.T
    span = f.ymax - f.ymin
    U = np.zeros_like(Y)
    nz = span > 0.0
    U[:, nz] = (Y[:, nz] - f.ymin[nz]) / span[nz]
    return scale * U
