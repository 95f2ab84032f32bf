"""Pins of the divergence's position gradient (Section 4, Theorem 4.3;
envelope gradients of Appendix B.6), squared Euclidean penalty, at eps = 2
where each EGW problem has one attractor:

* central finite differences of the divergence computed with converged
  solves, along random directions for x and for y;
* zero at isometric measures: SGW >= 0 with equality there (Theorem 4.3),
  so such a pair is a minimum and the gradient vanishes, although each of
  the three envelope gradients is far from zero.
The same two pins hold the weight gradients (sgw_grad_weights), along
directions tangent to the simplex, and the lifted penalty's versions."""
import numpy as np

from oracle import gw_oracle as O

EPS = 2.0


def _measure(rng, n, d):
    x = rng.standard_normal((n, d)) * np.array([1.0, 0.6, 0.3][:d])
    a = rng.dirichlet(np.ones(n) * 3)
    return x, a


def test_position_gradient_matches_finite_differences():
    rng = np.random.default_rng(40)
    x, a = _measure(rng, 9, 2)
    y, b = _measure(rng, 8, 2)
    gx, gy = O.sgw_grad_positions(a, b, x, y, EPS)
    h = 1e-5
    for _ in range(2):
        dx = rng.standard_normal(x.shape)
        dx /= np.linalg.norm(dx)
        fd = (O.sgw_value_converged(a, b, x + h * dx, y, EPS)
              - O.sgw_value_converged(a, b, x - h * dx, y, EPS)) / (2 * h)
        assert abs(fd - np.sum(gx * dx)) < 1e-6 * np.abs(gx).sum()
        dy = rng.standard_normal(y.shape)
        dy /= np.linalg.norm(dy)
        fd = (O.sgw_value_converged(a, b, x, y + h * dy, EPS)
              - O.sgw_value_converged(a, b, x, y - h * dy, EPS)) / (2 * h)
        assert abs(fd - np.sum(gy * dy)) < 1e-6 * np.abs(gy).sum()


def test_gradient_vanishes_between_isometric_measures():
    rng = np.random.default_rng(41)
    x, a = _measure(rng, 10, 2)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    perm = rng.permutation(10)
    y = (x @ R.T + np.array([0.3, -1.2]))[perm]
    b = a[perm]
    gx, gy = O.sgw_grad_positions(a, b, x, y, EPS)
    X, Y = O.centre(x, a), O.centre(y, b)
    gam, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, EPS)
    scale = np.abs(O.grad_positions_sqeuclid(X, Y, a, b, pi, gam)).max()
    assert scale > 1e-2
    assert np.abs(gx).max() < 1e-8 * scale and np.abs(gy).max() < 1e-8 * scale


# |x - x'| lifted by frozen landmark maps (Algorithm 4 and Algorithm 13):
# alpha is embedded by Pi_x and beta by Pi_y in every term of the divergence


def _lifted_case(rng, n, m, p=1.0, dim=4):
    x, a = _measure(rng, n, 2)
    y, b = _measure(rng, m, 2)
    lmx = O.fit_landmarks(x[: n - 2], p, dim)
    lmy = O.fit_landmarks(y[: m - 2], p, dim)
    return x, a, y, b, lmx, lmy


def test_lifted_gradient_matches_finite_differences():
    rng = np.random.default_rng(42)
    x, a, y, b, lmx, lmy = _lifted_case(rng, 9, 8)
    gx, gy = O.sgw_grad_positions_lifted(a, b, x, y, EPS, lmx, lmy)
    h = 1e-5
    for _ in range(2):
        dx = rng.standard_normal(x.shape)
        dx /= np.linalg.norm(dx)
        fd = (O.sgw_value_converged_lifted(a, b, x + h * dx, y, EPS, lmx, lmy)
              - O.sgw_value_converged_lifted(a, b, x - h * dx, y, EPS, lmx, lmy)) / (2 * h)
        assert abs(fd - np.sum(gx * dx)) < 1e-6 * np.abs(gx).sum()
        dy = rng.standard_normal(y.shape)
        dy /= np.linalg.norm(dy)
        fd = (O.sgw_value_converged_lifted(a, b, x, y + h * dy, EPS, lmx, lmy)
              - O.sgw_value_converged_lifted(a, b, x, y - h * dy, EPS, lmx, lmy)) / (2 * h)
        assert abs(fd - np.sum(gy * dy)) < 1e-6 * np.abs(gy).sum()


def test_lifted_gradient_of_the_linear_kernel_is_the_squared_norm_gradient():
    # p = 2 with D = d: the landmark kernel is linear and the map an isometry
    # of the plane onto its principal axes, so the lifted divergence is the
    # squared-norm one and so is its gradient
    rng = np.random.default_rng(43)
    x, a, y, b, lmx, lmy = _lifted_case(rng, 9, 8, p=2.0, dim=2)
    gx, gy = O.sgw_grad_positions_lifted(a, b, x, y, EPS, lmx, lmy)
    hx, hy = O.sgw_grad_positions(a, b, x, y, EPS)
    assert np.abs(gx - hx).max() < 1e-9 * np.abs(hx).max()
    assert np.abs(gy - hy).max() < 1e-9 * np.abs(hy).max()


def test_lifted_gradient_vanishes_between_isometric_measures():
    # y is a rigid motion of x (permuted) and beta's landmarks are the images
    # of alpha's in the same order: both maps see the same landmark kernel,
    # so the embedded measures coincide and the pair is a minimum
    rng = np.random.default_rng(44)
    x, a = _measure(rng, 10, 2)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    perm = rng.permutation(10)
    y = (x @ R.T + np.array([0.3, -1.2]))[perm]
    b = a[perm]
    lm_idx = np.arange(8)
    lmx = O.fit_landmarks(x[lm_idx], 1.0, 4)
    inv = np.argsort(perm)
    lmy = O.fit_landmarks(y[inv[lm_idx]], 1.0, 4)
    gx, gy = O.sgw_grad_positions_lifted(a, b, x, y, EPS, lmx, lmy)
    X, Y = O.landmark_features(x, a, lmx), O.landmark_features(y, b, lmy)
    gam, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, EPS)
    pair = np.einsum("nd,ndk->nk", O.chain_centre(O.grad_features(X, Y, a, b, pi, gam), a),
                     O.kernel_proj_jacobian(x, lmx))
    scale = np.abs(pair).max()
    assert scale > 1e-2
    assert np.abs(gx).max() < 1e-7 * scale and np.abs(gy).max() < 1e-7 * scale


# Weight gradients (sgw_grad_weights): each EGW problem's derivative along the
# simplex is the EOT potential of its linearised cost on that side, and
# GW_eps(alpha, alpha) carries a in both marginals


def _tangent(rng, w):
    u = rng.standard_normal(len(w))
    d = w * (u - w @ u)
    return d / np.linalg.norm(d)


def test_weight_gradient_matches_finite_differences():
    rng = np.random.default_rng(42)
    x, a = _measure(rng, 9, 2)
    y, b = _measure(rng, 8, 2)
    ga, gb = O.sgw_grad_weights(a, b, x, y, EPS)
    assert abs(a @ ga) < 1e-12 * np.abs(ga).max() and abs(b @ gb) < 1e-12 * np.abs(gb).max()
    h = 1e-5
    for _ in range(2):
        da = _tangent(rng, a)
        fd = (O.sgw_value_converged(a + h * da, b, x, y, EPS) - O.sgw_value_converged(a - h * da, b, x, y, EPS)) / (2 * h)
        assert abs(fd - ga @ da) < 1e-6 * np.abs(ga).sum()
        db = _tangent(rng, b)
        fd = (O.sgw_value_converged(a, b + h * db, x, y, EPS) - O.sgw_value_converged(a, b - h * db, x, y, EPS)) / (2 * h)
        assert abs(fd - gb @ db) < 1e-6 * np.abs(gb).sum()


def test_weight_gradient_vanishes_between_isometric_measures():
    # beta an isometric copy of alpha (SGW = 0, its minimum by Theorem 4.3):
    # moving either measure's weights along the simplex cannot lower it
    rng = np.random.default_rng(41)
    x, a = _measure(rng, 10, 2)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    perm = rng.permutation(10)
    y = (x @ R.T + np.array([0.3, -1.2]))[perm]
    b = a[perm]
    ga, gb = O.sgw_grad_weights(a, b, x, y, EPS)
    X, Y = O.centre(x, a), O.centre(y, b)
    _, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, EPS)
    scale = np.abs(O.grad_weights(O.sqdist(X, X), O.sqdist(Y, Y), a, b, pi, EPS)).max()
    assert scale > 1e-1
    assert np.abs(ga).max() < 1e-8 * scale and np.abs(gb).max() < 1e-8 * scale


def test_lifted_weight_gradient_matches_finite_differences():
    # |x - x'|^1.5 lifted to D = 4 by frozen maps (the weights also move the
    # re-centring of the features, which the squared distances do not see)
    rng = np.random.default_rng(44)
    x, a = _measure(rng, 9, 2)
    y, b = _measure(rng, 8, 2)
    lmx, lmy = O.fit_landmarks(x[:7], 1.5, 4), O.fit_landmarks(y[:6], 1.5, 4)
    tol = 1e-11
    ga, gb = O.sgw_grad_weights_lifted(a, b, x, y, EPS, lmx, lmy, tol=tol)
    h = 1e-5

    def val(aa, bb):
        return O.sgw_value_converged_lifted(aa, bb, x, y, EPS, lmx, lmy, tol)

    da, db = _tangent(rng, a), _tangent(rng, b)
    fd_a = (val(a + h * da, b) - val(a - h * da, b)) / (2 * h)
    fd_b = (val(a, b + h * db) - val(a, b - h * db)) / (2 * h)
    assert abs(fd_a - ga @ da) < 1e-6 * np.abs(ga).sum()
    assert abs(fd_b - gb @ db) < 1e-6 * np.abs(gb).sum()
