"""Pins of the oracle's pre-processing (Section II-A: z-score, PCA keeping
the n leading components, min-max to [0, 1]):

- scikit-learn's StandardScaler -> PCA(n) -> MinMaxScaler pipeline, an
  independent implementation (SVD of the centred data), after aligning each
  component's sign to the oracle's convention;
- properties that hold by construction: the standardised training columns
  have mean 0 and population variance 1; the projected training rows have a
  diagonal sample covariance equal to the leading eigenvalues; training rows
  land in [0, 1] with every component's minimum 0 and maximum 1; the fit
  does not depend on the order of the training rows;
- special cases: a constant column standardises to 0; components of
  decorrelated data with distinct variances are the coordinate axes.
"""
import numpy as np
import pytest

from oracle import preprocess as pp
from synthdata import gen_images


def images(n, seed):
    x, _ = gen_images(n, seed)
    return x / np.pi  # raw pixel intensities in [0, 1]


@pytest.mark.parametrize("n_comp", [2, 16, 64])
def test_matches_scikit_learn_pipeline(n_comp):
    sk = pytest.importorskip("sklearn")
    from sklearn.decomposition import PCA
    from sklearn.preprocessing import MinMaxScaler, StandardScaler
    X = images(600, 41)
    Xt = images(40, 42)
    f = pp.fit(X, n_comp)
    ours = pp.transform(f, X)
    ours_t = pp.transform(f, Xt)
    ss = StandardScaler().fit(X)
    pca = PCA(n_components=n_comp, svd_solver="full").fit(ss.transform(X))
    comps = pp.fix_signs(pca.components_)
    assert np.allclose(np.abs(comps), np.abs(f.components), atol=1e-9)
    assert np.allclose(comps, f.components, atol=1e-9)
    Y = ss.transform(X) @ comps.T
    mm = MinMaxScaler().fit(Y)
    assert np.allclose(mm.transform(Y), ours, atol=1e-9)
    assert np.allclose(mm.transform(ss.transform(Xt) @ comps.T), ours_t, atol=1e-9)
    assert np.allclose(pca.explained_variance_, f.eigvals[:n_comp], rtol=1e-9)


def test_construction_properties():
    X = images(500, 7)
    f = pp.fit(X, 20)
    Z = pp.zscore(X, f.mu, f.sigma)
    live = f.sigma > 0
    assert np.allclose(Z[:, live].mean(axis=0), 0.0, atol=1e-12)
    assert np.allclose((Z[:, live] ** 2).mean(axis=0), 1.0, atol=1e-12)
    Y = Z @ f.components.T
    cov = (Y.T @ Y) / (len(X) - 1)
    assert np.allclose(cov, np.diag(f.eigvals[:20]), atol=1e-9 * f.eigvals[0])
    U = pp.transform(f, X)
    assert np.allclose(U.min(axis=0), 0.0, atol=0) and np.allclose(U.max(axis=0), 1.0, atol=1e-15)
    assert np.all(np.diff(f.eigvals) <= 0)
    perm = np.random.default_rng(0).permutation(len(X))
    g = pp.fit(X[perm], 20)
    assert np.allclose(g.components, f.components, atol=1e-9)
    assert np.allclose(pp.transform(g, X), U, atol=1e-9)
    assert np.allclose(pp.transform(f, X, np.pi), np.pi * U)


def test_special_cases():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((400, 4)) * np.array([5.0, 1.0, 3.0, 0.0])  # last column constant
    X[:, 3] = 2.5
    f = pp.fit(X, 3)
    assert f.sigma[3] == 0.0
    assert np.all(pp.zscore(X, f.mu, f.sigma)[:, 3] == 0.0)
    # standardised, independent columns: the covariance is close to the
    # identity on the first three axes; the leading components stay inside
    # those axes and the constant column contributes nothing
    assert np.allclose(f.components[:, 3], 0.0, atol=1e-12)
    assert abs(f.eigvals[-1]) < 1e-12
    # a known rank-one structure: x = t * a + small noise -> component = a/|a|
    t = rng.standard_normal(1000)
    a = np.array([3.0, -1.0, 2.0])
    Y = np.outer(t, a) + 1e-6 * rng.standard_normal((1000, 3))
    g = pp.fit(Y, 1)
    w = np.sign(a) / np.sqrt(3.0)
    assert np.allclose(np.abs(g.components[0]), np.abs(w), atol=1e-5)
    assert g.components[0][np.argmax(np.abs(g.components[0]))] > 0


def test_planted_sign_convention_mistake_is_caught():
    """Flipping one component's sign mirrors that coordinate (u -> 1 - u):
    the scikit-learn pin sees it unless signs are aligned by the convention."""
    X = images(300, 11)
    f = pp.fit(X, 4)
    U = pp.transform(f, X)
    f.components[1] *= -1.0
    f.ymin[1], f.ymax[1] = -f.ymax[1], -f.ymin[1]
    V = pp.transform(f, X)
    assert np.allclose(V[:, 1], 1.0 - U[:, 1], atol=1e-12)
    assert not np.allclose(V, U, atol=1e-3)
