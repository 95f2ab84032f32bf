"""Full-N kernel PCA on the GPU (gw_kpca_full through the C ABI) against the
oracle's exact eigendecomposition of Algorithm 4's kernel.

Eigenvectors are unique only up to sign, so the comparison is on what is
unique: the eigenvalues and the Gram matrix of the features, X X^T =
V Lambda V^T (unique when the D-th eigenvalue is separated from the next).
Tolerances: the iteration shrinks the error of the D-th direction by about
(lambda_{D+32} / lambda_D)^(2 n_iter + 1), and the Rayleigh-Ritz step turns
it into an eigenvector error of that over the relative gap lambda_D /
lambda_{D+1} - 1 (2% at D = 64 here, hence 20 steps there); features are
stored in single precision.  Eigenvalues within 1e-6 of the largest, Gram
entries within 1e-5 of the largest.  At full rank (D = n - 1, where the
block spans the whole space) the features reproduce the cost itself."""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as O
from workloads import config3_scale

pytestmark = pytest.mark.gpu


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("n,p,D,n_iter", [(1500, 1.0, 16, 10), (1500, 1.0, 64, 20), (1100, 0.5, 32, 10),
                                           (900, 2.0, 8, 10)])
def test_kpca_matches_oracle(gw, n, p, D, n_iter):
    prob = config3_scale(n=n, lifted_dim=D)
    x = prob.x.astype(np.float32).astype(np.float64)
    a = prob.a.astype(np.float32).astype(np.float64)
    print(f"kpca n={n} p={p} D={D}", flush=True)
    X, lam = gw.Context().kpca_full(dev(x), dev(a), p=p, D=D, n_iter=n_iter, seed=3)
    X = X.cpu().numpy().astype(np.float64)
    Xo, lamo = O.full_kpca_features(x, a, p, D)
    lam = np.array(lam)
    keep = lamo > 1e-9 * lamo[0]
    print("lambda err", np.max(np.abs(lam[keep] - lamo[keep])) / lamo[0])
    assert np.max(np.abs(lam[keep] - lamo[keep])) <= 1e-6 * lamo[0]
    G, Go = X @ X.T, Xo @ Xo.T
    err = np.max(np.abs(G - Go)) / np.max(np.abs(Go))
    print("gram err", err)
    assert err <= 1e-5
    assert np.max(np.abs(a @ X)) <= 1e-5 * np.sqrt(lamo[0])


def test_kpca_full_rank_reproduces_cost(gw):
    rng = np.random.default_rng(5)
    n = 70
    x = rng.standard_normal((n, 2)).astype(np.float32).astype(np.float64)
    a = np.full(n, 1.0 / n)
    X, lam = gw.Context().kpca_full(dev(x), dev(a), p=1.0, D=n - 1, n_iter=2, seed=1)
    X = X.cpu().numpy().astype(np.float64)
    d2 = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    c = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    assert np.max(np.abs(d2 - c)) <= 1e-5 * c.max()


def test_kpca_rejects_bad_arguments(gw):
    x = dev(np.zeros((10, 3)) + np.arange(10)[:, None])
    a = dev(np.full(10, 0.1))
    ctx = gw.Context()
    for kw in (dict(p=0.0), dict(p=2.5), dict(D=10), dict(D=0), dict(n_iter=-1)):
        with pytest.raises(gw.GWError):
            ctx.kpca_full(x, a, **{"D": 4, **kw})
    with pytest.raises(gw.GWError):
        ctx.kpca_full(dev(np.zeros((10, 9))), a, D=4)
