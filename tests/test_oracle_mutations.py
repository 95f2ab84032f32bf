"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins catch them.  Each mutation is undone by monkeypatch after its test."""
import numpy as np

from oracle import gw_oracle as O


def _pair(seed=40, n=6, m=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 2))
    y = rng.standard_normal((m, 2))
    a = rng.dirichlet(np.ones(n) * 2)
    b = rng.dirichlet(np.ones(m) * 2)
    return rng, x, a, y, b


def _p4_gap():
    _, x, a, y, b = _pair()
    X, Y = O.centre(x, a), O.centre(y, b)
    res = O.cnt_gw(a, b, X, Y, 0.3, 0.3, 2, 0, record=True, inner_tol=1e-14)
    egw = O.entropic_gw(a, b, O.sqdist(x, x), O.sqdist(y, y), 0.3, 2, 0, inner_tol=1e-14)
    return max(np.abs(res.history[t]["pi"] - egw[t]).max() for t in range(2))


def _p1_gap():
    rng, x, a, y, b = _pair()
    X, Y = O.centre(x, a), O.centre(y, b)
    c = rng.standard_normal((len(a), len(b)))
    f, g = O.sinkhorn_converged(a, b, c, 0.5)
    pi = O.plan(a, b, f, g, c, 0.5)
    return abs(O.lifted_loss(X, Y, a, b, pi) - O.quartic_loss(O.sqdist(x, x), O.sqdist(y, y), pi))


def test_unmutated_pins_pass():
    assert _p4_gap() < 1e-12
    assert _p1_gap() < 1e-10


def test_wrong_lift_half_is_caught(monkeypatch):
    monkeypatch.setattr(O, "lift", lambda v: np.concatenate([v, np.sum(v * v, 1, keepdims=True)], 1))
    assert _p4_gap() > 1e-4


def test_wrong_temperature_is_caught(monkeypatch):
    real = O.sinkhorn
    monkeypatch.setattr(O, "sinkhorn_converged",
                        lambda a, b, c, eps, f0=None, g0=None, tol=1e-14, **kw:
                        real(a, b, c, eps * 8 if eps < 0.1 else eps, 4000, f0, g0))
    assert _p4_gap() > 1e-4


def test_wrong_covariance_factor_is_caught(monkeypatch):
    real = O.lifted_loss

    def bad(X, Y, a, b, pi):
        gam = X.T @ pi @ Y
        return real(X, Y, a, b, pi) + 4.0 * float(np.sum(gam * gam))
    monkeypatch.setattr(O, "lifted_loss", bad)
    assert _p1_gap() > 1e-4


def test_dropped_gradient_term_is_caught(monkeypatch):
    rng, x, a, y, b = _pair(41)
    X, Y = O.centre(x, a), O.centre(y, b)
    gam, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, 0.5)
    good = O.grad_positions_sqeuclid(X, Y, a, b, pi, gam)
    quart = O.grad_positions_quartic(x, a, pi, O.sqdist(y, y))
    assert np.abs(good - quart).max() < 1e-9
    real = O.grad_features
    monkeypatch.setattr(O, "grad_features",
                        lambda X, Y, a, b, pi, gamma: real(X, Y, a, b, pi, gamma)
                        + 8.0 * X * (pi @ np.sum(Y * Y, 1))[:, None])
    bad = O.grad_positions_sqeuclid(X, Y, a, b, pi, gam)
    assert np.abs(bad - quart).max() > 1e-3
