"""Pins of the divergence's position gradient (Section 4, Theorem 4.3;
envelope gradients of Appendix B.6), squared Euclidean penalty, at eps = 2
where each EGW problem has one attractor:

* central finite differences of the divergence computed with converged
  solves, along random directions for x and for y;
* zero at isometric measures: SGW >= 0 with equality there (Theorem 4.3),
  so such a pair is a minimum and the gradient vanishes, although each of
  the three envelope gradients is far from zero."""
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
