"""Pins of the multiscale oracle (Appendix B, Multiscale-GW: Coarsen,
Algorithm 8 Interpolate, Algorithm 7) against facts that do not come from
the oracle itself: a Lloyd iteration worked by hand, scikit-learn's K-Means
on the same start, the textbook float64 Lloyd iteration (kmeans_plain) of
which coarsen is the fixed-point form, exact identities (one point per cluster, conservation of
weight and mean), the paper's own bilinear form of Algorithm 8 evaluated
with scipy's logsumexp, the Sinkhorn fixed point, and the fixed point of
Algorithm 1 carried from the coarse to the fine scale."""
import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import gw_oracle as O
from workloads import synth


def _gmm(rng, n, d, k=4, sigma=0.05):
    means = rng.uniform(-1, 1, size=(k, d))
    lab = rng.integers(0, k, size=n)
    return means[lab] + sigma * rng.standard_normal((n, d))


def test_lloyd_worked_example():
    # points 0, 1, 10, 11 with weights .1 .2 .3 .4, started at the first two:
    # step 1 assigns {0} and {1, 10, 11} (centroid 7.6 / .9); step 2 moves 1
    # to the first cluster: centroids (.2 / .3) and (3 + 4.4) / .7, stable after.
    X = np.array([[0.0], [1.0], [10.0], [11.0]])
    a = np.array([0.1, 0.2, 0.3, 0.4])
    Xc, ac, assign, kept = O.coarsen(X, a, [0, 1], 1)
    assert list(assign) == [0, 1, 1, 1]
    assert Xc[1, 0] == np.float32(7.6 / 0.9)
    Xc, ac, assign, kept = O.coarsen(X, a, [0, 1], 4)
    assert list(assign) == [0, 0, 1, 1] and list(kept) == [0, 1]
    assert Xc[0, 0] == np.float32(2.0 / 3.0) and Xc[1, 0] == np.float32(74.0 / 7.0)
    # the cluster weights are exact sums of the single-precision weights
    w = a.astype(np.float32).astype(np.float64)
    assert ac[0] == np.float32(w[0] + w[1]) and ac[1] == np.float32(w[2] + w[3])


def test_one_point_per_cluster_is_exact():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((300, 7)).astype(np.float32)
    a = rng.dirichlet(np.ones(300)).astype(np.float32)
    perm = synth.splitmix64_landmarks(300, 300, 5)
    Xc, ac, assign, kept = O.coarsen(X, a, perm, 3)
    assert np.array_equal(Xc, X[perm])
    assert np.array_equal(ac, a[perm])
    inv = np.empty(300, np.int64)
    inv[perm] = np.arange(300)
    assert np.array_equal(assign, inv)


def test_matches_scikit_learn_lloyd():
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(2)
    X = _gmm(rng, 2000, 3, k=12, sigma=0.03).astype(np.float32)
    a = rng.uniform(0.5, 1.5, 2000)
    a = (a / a.sum()).astype(np.float32)
    init = synth.splitmix64_landmarks(2000, 40, 9)
    Xc, ac, assign, kept = O.coarsen(X, a, init, 100)
    km = KMeans(n_clusters=40, init=X[init].astype(np.float64), n_init=1, max_iter=100, tol=0.0,
                algorithm="lloyd").fit(X.astype(np.float64), sample_weight=a.astype(np.float64))
    assert len(kept) == 40
    assert np.array_equal(assign, km.labels_)
    assert np.max(np.abs(Xc - km.cluster_centers_)) < 1e-6


def test_conservation_and_empty_clusters():
    rng = np.random.default_rng(3)
    X = _gmm(rng, 1500, 5).astype(np.float32)
    a = rng.dirichlet(np.ones(1500)).astype(np.float32)
    init = list(synth.splitmix64_landmarks(1500, 60, 4))
    init[7] = init[3]        # a duplicated start: the later copy loses every tie and empties
    Xc, ac, assign, kept = O.coarsen(X, a, init, 1)
    assert 7 not in kept and len(kept) <= 59 and len(Xc) == len(kept)
    assert set(np.unique(assign)) == set(kept)
    Xc, ac, assign, kept = O.coarsen(X, a, init, 6)
    assert set(np.unique(assign)) == set(kept)
    a64 = a.astype(np.float64)
    assert abs(ac.astype(np.float64).sum() - a64.sum()) < 1e-6
    # sum_c ac Xc = sum_i a_i X_i up to the single-precision centroids
    lhs = (ac.astype(np.float64)[:, None] * Xc.astype(np.float64)).sum(0)
    rhs = (a64[:, None] * X.astype(np.float64)).sum(0)
    assert np.max(np.abs(lhs - rhs)) < 1e-6


def test_nearest_ties_go_to_lowest_index():
    X = np.array([[0.0, 0.0], [1.0, 1.0]], np.float32)
    C = np.array([[2.0, 2.0], [0.5, 0.5], [0.5, 0.5], [0.0, 0.0]], np.float32)
    assert list(O.nearest_centroid(X, C, block=1)) == [3, 1]
    assert list(O.nearest_centroid(X, C, block=256)) == [3, 1]


def _dyadic_weights(rng, n):
    """Weights k / 2^20 summing to exactly 1: single precision holds them
    exactly, so the coarse masses stay balanced."""
    k = np.floor(rng.dirichlet(np.ones(n) * 5) * 2 ** 20).astype(np.int64)
    k[-1] += 2 ** 20 - k.sum()
    return k / 2.0 ** 20


def _problem(rng, n, m, dx, dy):
    X = O.centre(rng.standard_normal((n, dx)), np.full(n, 1.0 / n))
    Y = O.centre(rng.standard_normal((m, dy)), np.full(m, 1.0 / m))
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    return X, Y, a, b


def test_interpolate_one_coarse_point_closed_form():
    rng = np.random.default_rng(4)
    P = rng.standard_normal((9, 3))
    Q = rng.standard_normal((1, 2))
    G = rng.standard_normal((3, 2))
    h = np.array([0.37])
    f = O.interpolate(h, P, Q, np.array([1.0]), G, 0.2, side=0)
    z = G @ Q[0]
    dist = np.sum((P - z) ** 2, 1) + (0.5 * np.sum(P * P, 1) - 0.5 * np.sum(Q[0] ** 2)) ** 2
    assert np.allclose(f, dist - h[0], atol=1e-12)


@pytest.mark.parametrize("side", [0, 1])
def test_interpolate_is_the_papers_bilinear_form(side):
    # Algorithm 8 as printed: C_ij = -4 |X_i|^2 |Y_j|^2 - 16 X_i^T Gamma Y_j at
    # temperature eps, with potentials in the bilinear convention F = 8 (f - alpha).
    rng = np.random.default_rng(5 + side)
    n, m, D, E, eps = 40, 11, 4, 3, 0.3
    X = rng.standard_normal((n, D))
    Y = rng.standard_normal((m, E))
    G = rng.standard_normal((D, E))
    w = rng.dirichlet(np.ones(m if side == 0 else n))
    if side == 0:
        h = rng.standard_normal(m)
        out = O.interpolate(h, X, Y, w, G, eps, side=0)
        nx, my = np.sum(X * X, 1), np.sum(Y * Y, 1)
        alpha = nx + nx ** 2 / 4
        beta = np.sum((Y @ G.T) ** 2, 1) + my ** 2 / 4
        C = -4 * nx[:, None] * my[None, :] - 16 * X @ G @ Y.T
        H = 8 * (h - beta)
        F = -eps * logsumexp(np.log(w)[None, :] + (H[None, :] - C) / eps, axis=1)
        assert np.allclose(out, alpha + F / 8, rtol=0, atol=1e-10 * (1 + np.abs(out).max()))
    else:
        h = rng.standard_normal(n)
        out = O.interpolate(h, Y, X, w, G, eps, side=1)
        nx, my = np.sum(X * X, 1), np.sum(Y * Y, 1)
        alpha = nx + nx ** 2 / 4
        beta = np.sum((Y @ G.T) ** 2, 1) + my ** 2 / 4
        C = -4 * nx[:, None] * my[None, :] - 16 * X @ G @ Y.T
        H = 8 * (h - alpha)
        F = -eps * logsumexp(np.log(w)[:, None] + (H[:, None] - C) / eps, axis=0)
        assert np.allclose(out, beta + F / 8, rtol=0, atol=1e-10 * (1 + np.abs(out).max()))


def test_interpolate_keeps_a_sinkhorn_fixed_point():
    rng = np.random.default_rng(6)
    X, Y, a, b = _problem(rng, 30, 25, 3, 2)
    G = 0.3 * rng.standard_normal((3, 2))
    eps = 0.4
    C = O.sqdist(O.lift(X), O.target_lift(Y, G))
    f, g = O.sinkhorn_converged(a, b, C, eps / 8, tol=1e-14)
    assert np.allclose(O.interpolate(g, X, Y, b, G, eps, side=0), f, atol=1e-10)
    assert np.allclose(O.interpolate(f, Y, X, a, G, eps, side=1), g, atol=1e-10)


def test_msgw_carries_a_converged_coarse_solution():
    # With one point per cluster the coarse problem is the fine one, permuted.
    # Once the coarse solve has reached a fixed point of Algorithm 1,
    # interpolation returns its potentials and the fine solve stays there.
    rng = np.random.default_rng(7)
    n, m = 24, 20
    X, Y, a, b = _problem(rng, n, m, 2, 2)
    X, Y = 0.5 * X, 0.5 * Y
    a = _dyadic_weights(rng, n)
    b = _dyadic_weights(rng, m)
    X, Y = O.centre(X, a), O.centre(Y, b)
    px = synth.splitmix64_landmarks(n, n, 1)
    py = synth.splitmix64_landmarks(m, m, 2)
    eps = 0.5
    coarse = dict(eps_start=eps, eps_end=eps, n_outer=150, n_inner=0, inner_tol=1e-14)
    fine = dict(eps_start=eps, eps_end=eps, n_outer=3, n_inner=0, inner_tol=1e-14)
    r = O.msgw(a, b, X, Y, px, py, 2, coarse, fine)
    ref = O.cnt_gw(a, b, X, Y, eps, eps, 150, 0, inner_tol=1e-14)
    # the coarse solve is the fine problem with rows and columns permuted
    # (its features rounded to single precision: differences of order 1e-7)
    assert np.allclose(r.coarse.gamma, ref.gamma, atol=1e-6)
    assert np.allclose(r.f0, ref.f, atol=1e-6) and np.allclose(r.g0, ref.g, atol=1e-6)
    assert np.allclose(r.fine.gamma, ref.gamma, atol=1e-7)
    lf = O.egw_objective(X, Y, a, b, r.fine.pi, eps)
    lr = O.egw_objective(X, Y, a, b, ref.pi, eps)
    assert abs(lf - lr) < 1e-7 * abs(lr)


def test_msgw_invariant_under_rotation_of_one_side():
    rng = np.random.default_rng(8)
    n, m = 300, 260
    X = _gmm(rng, n, 3, k=5)
    Y = _gmm(rng, m, 3, k=5)
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    R = q * np.sign(np.diag(r))
    px = synth.splitmix64_landmarks(n, 30, 1)
    py = synth.splitmix64_landmarks(m, 26, 2)
    sched = dict(eps_start=0.1, eps_end=0.1, n_outer=8, n_inner=40)
    r1 = O.msgw(a, b, X, Y, px, py, 5, sched, sched)
    r2 = O.msgw(a, b, X, Y @ R.T, px, py, 5, sched, sched)
    l1 = O.egw_objective(O.centre(X, a), O.centre(Y, b), a, b, r1.fine.pi, 0.1)
    l2 = O.egw_objective(O.centre(X, a), O.centre(Y @ R.T, b), a, b, r2.fine.pi, 0.1)
    assert abs(l1 - l2) <= 1e-5 * abs(l1)


def test_coarsen_is_plain_kmeans_away_from_ties():
    # coarsen fixes the precision of the sums (a 2^-S grid) and of the
    # distances (single precision); on generic inputs, where no assignment
    # falls within that rounding of a tie, it is the float64 textbook
    # algorithm: the same assignments and kept clusters, the cluster weights
    # and centroids to single precision
    rng = np.random.default_rng(11)
    for trial in range(4):
        X = _gmm(rng, 400, 3, k=6, sigma=0.08).astype(np.float32)
        a = rng.dirichlet(np.ones(400) * 2).astype(np.float32)
        init = rng.choice(400, size=12, replace=False)
        Xc, ac, assign, kept = O.coarsen(X, a, init, 5)
        C, w, assign_p = O.kmeans_plain(X, a, init, 5)
        assert np.array_equal(assign, assign_p), trial
        assert np.array_equal(kept, np.nonzero(w > 0)[0])
        assert np.allclose(ac, w[kept], rtol=1e-6, atol=0)
        assert np.abs(Xc - C[kept]).max() <= 4e-7 * np.abs(C).max()
