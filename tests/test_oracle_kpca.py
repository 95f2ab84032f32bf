"""Pins of the full-N kernel PCA oracle (Appendix B, "Kernel PCA" with
Algorithm 4): at full rank the features reproduce the CNT cost exactly
(|X_i - X_j|^2 = |x_i - x_j|^p, the defining property of the kernel of a
CNT cost), they are centred with the weights, and for p = 2 they are the
weighted PCA coordinates (numpy's SVD of the centred points)."""
import numpy as np
import pytest

from oracle import gw_oracle as O


@pytest.mark.parametrize("p", [0.5, 1.0, 2.0])
def test_full_rank_features_reproduce_the_cost(p):
    rng = np.random.default_rng(int(10 * p))
    n = 40
    x = rng.standard_normal((n, 3))
    a = rng.dirichlet(np.ones(n) * 3)
    X, lam = O.full_kpca_features(x, a, p, n - 1)
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    c = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)) ** p
    assert np.max(np.abs(d2 - c)) < 1e-9 * c.max()
    assert np.max(np.abs(a @ X)) < 1e-10
    assert np.all(np.diff(lam) <= 1e-12)


def test_squared_norm_gives_weighted_pca():
    rng = np.random.default_rng(3)
    n = 60
    x = rng.standard_normal((n, 3)) * np.array([2.0, 1.0, 0.3])
    a = np.full(n, 1.0 / n)
    X, lam = O.full_kpca_features(x, a, 2.0, 3)
    xc = x - x.mean(0)
    u, sv, vt = np.linalg.svd(xc, full_matrices=False)
    pca = xc @ vt.T
    assert np.allclose(lam, sv ** 2, rtol=1e-10)
    assert np.allclose(np.abs(X), np.abs(pca), atol=1e-10)
