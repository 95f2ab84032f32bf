"""Pins of the oracle's lifting of CNT penalties into features.

P11: with every point a landmark and full rank, kernel PCA reproduces the
cost exactly (Schoenberg: c(x, x') = |phi(x) - phi(x')|^2); the Nystrom map
(Algorithm 13) reproduces the landmarks' own features; centring makes
sum_i a_i X_i = 0.  Algorithm 4's centring makes the kernel independent of
the base point.
"""
import numpy as np
import pytest

from oracle import gw_oracle as O
from workloads import landmark_indices


@pytest.mark.parametrize("p", [1.0, 0.5, 1.5, 2.0])
def test_full_rank_kpca_is_exact(p):
    rng = np.random.default_rng(20)
    x = rng.standard_normal((40, 3))
    lm = O.fit_landmarks(x, p, 40)
    X = O.kernel_proj(x, lm)
    c = O.power_cost(x, x, p)
    assert np.abs(O.sqdist(X, X) - c).max() < 1e-10 * max(1.0, c.max())


def test_kernel_psd_for_cnt_and_not_for_p3():
    """CNT (p <= 2) gives a positive semi-definite centred kernel; p = 3 is
    outside the class and does not (Section 2, Embeddable Costs)."""
    rng = np.random.default_rng(21)
    x = rng.standard_normal((30, 2))
    w = np.full(30, 1 / 30)
    for p, psd in ((1.0, True), (2.0, True), (3.0, False)):
        lam = np.linalg.eigvalsh(O.kernel_from_cost(O.power_cost(x, x, p), w))
        assert (lam.min() > -1e-10 * lam.max()) == psd


def test_kernel_independent_of_base_point():
    rng = np.random.default_rng(22)
    x = rng.standard_normal((12, 3))
    w = rng.dirichlet(np.ones(12))
    c = O.power_cost(x, x, 1.0)
    k1 = O.kernel_from_cost(c, w)
    perm = np.roll(np.arange(12), 5)
    k2 = O.kernel_from_cost(c[np.ix_(perm, perm)], w[perm])
    assert np.abs(k1[np.ix_(perm, perm)] - k2).max() < 1e-12
    # weighted centring: sum_i w_i K_ij = 0
    assert np.abs(w @ k1).max() < 1e-12


def test_nystrom_reproduces_landmarks_and_centres():
    rng = np.random.default_rng(23)
    x = rng.standard_normal((300, 3))
    a = rng.dirichlet(np.ones(300))
    idx = landmark_indices(300, 64, seed=5)
    lm = O.fit_landmarks(x[idx], 1.0, 16)
    pix = O.kernel_proj(x[idx], lm)
    assert np.abs(pix - lm.vec * np.sqrt(lm.lam)[None, :]).max() < 1e-10
    X = O.landmark_features(x, a, lm)
    assert np.abs(a @ X).max() < 1e-14
    # truncated embedding: distances are approximated, never exceeded by
    # much more than the discarded spectrum
    c = O.power_cost(x[idx], x[idx], 1.0)
    err = np.abs(O.sqdist(pix, pix) - c).max()
    assert err < 0.5 * c.max()


def test_jacobian_matches_finite_differences():
    rng = np.random.default_rng(24)
    pts = rng.standard_normal((50, 3))
    lm = O.fit_landmarks(pts, 1.0, 12)
    x = rng.standard_normal((7, 3))
    jac = O.kernel_proj_jacobian(x, lm)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (O.kernel_proj(x + e, lm) - O.kernel_proj(x - e, lm)) / (2 * h)
        assert np.abs(fd - jac[:, :, k]).max() < 1e-6


def test_landmark_choice_is_seeded_prefix():
    idx = landmark_indices(1000, 50, seed=3)
    want = np.sort(np.random.default_rng(3).permutation(1000)[:50])
    assert np.array_equal(idx, want)
    assert np.array_equal(landmark_indices(10, 50, seed=3), np.arange(10))
