"""Pins of the oracle's gradients (Appendix B.6).

* The lifted-form envelope gradient equals the envelope gradient of the
  quartic GW loss itself (independent algebra, no features).
* Both equal central finite differences of a converged solve (the EGW value
  as a function of the inputs), for the squared-Euclidean penalty and for the
  |x - x'| penalty lifted through frozen landmarks.
* Invariants: translation (sum_i G_i = 0) and rotation (sum_i G_i x_i^T
  symmetric).
* Weight gradient: the Lagrange potential of the linearised problem against
  finite differences along directions tangent to the simplex.
"""
import numpy as np
import pytest

from oracle import gw_oracle as O

EPS = 0.5


def _problem(seed, n=9, m=8, d=2):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    y = 0.8 * rng.standard_normal((m, d))
    a = rng.dirichlet(np.ones(n) * 3)
    b = rng.dirichlet(np.ones(m) * 3)
    return rng, x, a, y, b


def _solve_sq(x, a, y, b, gamma0=None):
    X, Y = O.centre(x, a), O.centre(y, b)
    gam, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, EPS, gamma0=gamma0)
    return X, Y, gam, pi, O.egw_objective(X, Y, a, b, pi, EPS)


def test_lifted_gradient_equals_quartic_envelope():
    _, x, a, y, b = _problem(30)
    X, Y, gam, pi, _ = _solve_sq(x, a, y, b)
    g_lift = O.grad_positions_sqeuclid(X, Y, a, b, pi, gam)
    g_quart = O.grad_positions_quartic(x, a, pi, O.sqdist(y, y))
    assert np.abs(g_lift - g_quart).max() < 1e-9 * np.abs(g_lift).max()


def test_position_gradient_finite_differences():
    rng, x, a, y, b = _problem(31)
    X, Y, gam, pi, _ = _solve_sq(x, a, y, b)
    grad = O.grad_positions_sqeuclid(X, Y, a, b, pi, gam)
    h = 1e-4
    for _ in range(4):
        d = rng.standard_normal(x.shape)
        d /= np.linalg.norm(d)
        lp = _solve_sq(x + h * d, a, y, b, gam)[4]
        lm = _solve_sq(x - h * d, a, y, b, gam)[4]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.sum(grad * d)) < 1e-6 * max(1.0, abs(fd))


def test_target_gradient_finite_differences():
    rng, x, a, y, b = _problem(32)
    X, Y, gam, pi, _ = _solve_sq(x, a, y, b)
    grad_y = O.chain_centre(O.grad_features_target(X, Y, a, b, pi, gam), b)
    h = 1e-4
    d = rng.standard_normal(y.shape)
    d /= np.linalg.norm(d)
    fd = (_solve_sq(x, a, y + h * d, b, gam)[4] - _solve_sq(x, a, y - h * d, b, gam)[4]) / (2 * h)
    assert abs(fd - np.sum(grad_y * d)) < 1e-6 * max(1.0, abs(fd))


def test_gradient_invariants():
    _, x, a, y, b = _problem(33)
    X, Y, gam, pi, _ = _solve_sq(x, a, y, b)
    g = O.grad_positions_sqeuclid(X, Y, a, b, pi, gam)
    assert np.abs(g.sum(0)).max() < 1e-12 * np.abs(g).max() * len(x)
    mom = g.T @ x
    assert np.abs(mom - mom.T).max() < 1e-10 * np.abs(mom).max()


def test_power_penalty_gradient_finite_differences():
    """|x - x'| penalty lifted through frozen landmarks (Algorithm 12 with
    Algorithm 13): the function x -> features -> converged EGW value."""
    rng = np.random.default_rng(34)
    n, m = 10, 9
    x = rng.standard_normal((n, 3))
    y = rng.standard_normal((m, 3))
    a = rng.dirichlet(np.ones(n) * 3)
    b = rng.dirichlet(np.ones(m) * 3)
    lmx = O.fit_landmarks(rng.standard_normal((30, 3)), 1.0, 8)
    lmy = O.fit_landmarks(rng.standard_normal((30, 3)), 1.0, 8)
    Y = O.landmark_features(y, b, lmy)

    def solve(xx, g0=None):
        X = O.landmark_features(xx, a, lmx)
        gam, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, EPS, gamma0=g0)
        return X, gam, pi, O.egw_objective(X, Y, a, b, pi, EPS)

    X, gam, pi, _ = solve(x)
    grad = O.grad_positions_power(x, X, Y, a, b, pi, gam, lmx)
    h = 1e-5
    for _ in range(3):
        d = rng.standard_normal(x.shape)
        d /= np.linalg.norm(d)
        fd = (solve(x + h * d, gam)[3] - solve(x - h * d, gam)[3]) / (2 * h)
        assert abs(fd - np.sum(grad * d)) < 1e-5 * max(1.0, abs(fd))


def test_weight_gradient_finite_differences():
    rng, x, a, y, b = _problem(35)
    X, Y, gam, pi, _ = _solve_sq(x, a, y, b)
    F = O.grad_weights(O.sqdist(X, X), O.sqdist(Y, Y), a, b, pi, EPS)
    h = 1e-5
    for _ in range(3):
        u = rng.standard_normal(len(a))
        da = a * (u - a @ u)
        da /= np.linalg.norm(da)
        fd = (_solve_sq(x, a + h * da, y, b, gam)[4] - _solve_sq(x, a - h * da, y, b, gam)[4]) / (2 * h)
        assert abs(fd - F @ da) < 1e-5 * max(1.0, abs(fd))
