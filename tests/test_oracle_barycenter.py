"""Pins of the GW barycentre flow (Section 6, "GW Barycenters") in the
oracle: with small steps the objective decreases at every step, and the
first decrease matches its first-order prediction step * sum_i |g_i|^2 / w_i
(which fixes the scaling of the update by the point weights)."""
import numpy as np

from oracle import gw_oracle as O

EPS = 2.0


def _clouds():
    rng = np.random.default_rng(60)
    x = rng.standard_normal((7, 2)) * np.array([1.0, 0.4])
    y = rng.standard_normal((6, 2)) * np.array([0.5, 0.9])
    a = np.full(7, 1.0 / 7)
    b = np.full(6, 1.0 / 6)
    z0 = rng.standard_normal((5, 2)) * 0.7
    w = np.full(5, 1.0 / 5)
    return a, b, x, y, z0, w


def test_flow_descends():
    a, b, x, y, z0, w = _clouds()
    _, obj = O.sgw_barycenter(a, b, x, y, z0, w, 0.3, 0.02, 3, EPS, tol=1e-10)
    assert all(obj[i + 1] < obj[i] for i in range(3))


def test_first_decrease_matches_first_order():
    a, b, x, y, z0, w = _clouds()
    lam, step = 0.3, 1e-5
    gzx, _ = O.sgw_grad_positions(w, a, z0, x, EPS, tol=1e-10)
    gzy, _ = O.sgw_grad_positions(w, b, z0, y, EPS, tol=1e-10)
    g = (1 - lam) * gzx + lam * gzy
    predicted = step * np.sum(g * g / w[:, None])
    _, obj = O.sgw_barycenter(a, b, x, y, z0, w, lam, step, 1, EPS, tol=1e-10)
    assert abs((obj[0] - obj[1]) - predicted) < 1e-3 * predicted


# |x - x'|^p lifted by frozen landmark maps, one per measure (z's landmark
# points stay where they were fitted while z moves).  p = 1.5: for p <= 1
# the penalty has a kink at zero distance, and the points that are
# landmarks start on it, where a one-sided step sees a first-order increase
# that the (sub)gradient 0 there does not predict.


def _lifted_maps(x, y, z0, p=1.5):
    return (O.fit_landmarks(z0, p, 3), O.fit_landmarks(x[:6], p, 3), O.fit_landmarks(y[:5], p, 3))


def test_lifted_flow_descends():
    a, b, x, y, z0, w = _clouds()
    lmz, lma, lmb = _lifted_maps(x, y, z0)
    _, obj = O.sgw_barycenter_lifted(a, b, x, y, z0, w, 0.3, 0.02, 3, EPS, lmz, lma, lmb, tol=1e-10)
    assert all(obj[i + 1] < obj[i] for i in range(3))


def test_lifted_first_decrease_matches_first_order():
    # |z - z_l|^1.5 has a curvature singularity at the landmarks, where the
    # points start, so the Taylor remainder of a step s is O(s^1.5) there:
    # the first-order prediction holds to 1e-3 at s = 1e-7 (3e-3 at 1e-5)
    a, b, x, y, z0, w = _clouds()
    lmz, lma, lmb = _lifted_maps(x, y, z0)
    lam, step = 0.3, 1e-7
    gzx, _ = O.sgw_grad_positions_lifted(w, a, z0, x, EPS, lmz, lma, tol=1e-12)
    gzy, _ = O.sgw_grad_positions_lifted(w, b, z0, y, EPS, lmz, lmb, tol=1e-12)
    g = (1 - lam) * gzx + lam * gzy
    predicted = step * np.sum(g * g / w[:, None])
    _, obj = O.sgw_barycenter_lifted(a, b, x, y, z0, w, lam, step, 1, EPS, lmz, lma, lmb, tol=1e-12)
    assert abs((obj[0] - obj[1]) - predicted) < 1e-3 * predicted
