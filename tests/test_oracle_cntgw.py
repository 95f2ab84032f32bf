"""Pins of the oracle's CNT-GW outer loop (Algorithm 1).

P4  three algorithms from different parts of the paper produce the same
    couplings when the inner Sinkhorn is converged: CNT-GW (Algorithm 1),
    Entropic-GW with grad L = 2 sum (cX - cY)^2 pi (primal-descent
    proposition) and Kernel-GW (Algorithm 5).
P5  permutation enumeration: the GW loss is concave on Pi(a, b) for CNT
    costs, so its minimum is at a permutation; annealed CNT-GW reaches it.
P6  rigid-motion invariance of the target.
P7  isometric inputs: the unregularised loss of the solution goes to 0.
P8  monotone EGW objective (primal descent) and the Theorem 4.5 bound.
P10 large eps: pi -> a x b and Gamma -> 0.
"""
import itertools

import numpy as np
import pytest

from oracle import gw_oracle as O


def _cloud(seed, n, d, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng, scale * rng.uniform(-1, 1, (n, d))


@pytest.mark.parametrize("symmetric", [True, False])
def test_cntgw_matches_entropic_gw_and_kernel_gw(symmetric):
    rng = np.random.default_rng(10)
    n, m = 7, 6
    x = rng.standard_normal((n, 2))
    y = rng.standard_normal((m, 3))
    a = rng.dirichlet(np.ones(n) * 2)
    b = rng.dirichlet(np.ones(m) * 2)
    X, Y = O.centre(x, a), O.centre(y, b)
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    eps = 0.3
    res = O.cnt_gw(a, b, X, Y, eps, eps, 4, 0, symmetric=symmetric, record=True,
                   inner_tol=1e-14)
    egw = O.entropic_gw(a, b, cx, cy, eps, 4, 0, inner_tol=1e-14)
    kgw = O.kernel_gw(a, b, cx, cy, eps, 4, 0, inner_tol=1e-14)
    for t in range(4):
        assert np.abs(res.history[t]["pi"] - egw[t]).max() < 1e-12
        assert np.abs(res.history[t]["pi"] - kgw[t]).max() < 1e-12


def test_entropic_gw_without_factor_two_differs():
    """The linearisation without the factor 2 is EOT at twice the
    temperature; it must not match CNT-GW (the reading of the factor)."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal((6, 2))
    y = rng.standard_normal((6, 2))
    a = np.full(6, 1 / 6)
    b = np.full(6, 1 / 6)
    X, Y = O.centre(x, a), O.centre(y, b)
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    eps = 0.2
    res = O.cnt_gw(a, b, X, Y, eps, eps, 2, 3000, record=True)
    pi = np.outer(a, b)
    for _ in range(2):
        c = 0.5 * O.full_linearisation(cx, cy, pi)
        f, g = O.sinkhorn(a, b, c, eps, 3000)
        pi = O.plan(a, b, f, g, c, eps)
    assert np.abs(res.history[1]["pi"] - pi).max() > 1e-3


def test_permutation_enumeration():
    n = 5
    rng, x = _cloud(12, n, 2)
    _, y = _cloud(13, n, 2)
    a = np.full(n, 1 / n)
    b = np.full(n, 1 / n)
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    best = np.inf
    for perm in itertools.permutations(range(n)):
        pi = np.zeros((n, n))
        pi[np.arange(n), perm] = 1 / n
        best = min(best, O.quartic_loss(cx, cy, pi))
    # concavity: every feasible plan is at least the best vertex
    for s in range(20):
        c = rng.standard_normal((n, n)) * 3
        f, g = O.sinkhorn_converged(a, b, c, 0.3, tol=1e-14)
        assert O.quartic_loss(cx, cy, O.plan(a, b, f, g, c, 0.3)) >= best - 1e-12
    # annealed CNT-GW from several random Gamma_0 reaches the minimum; the
    # start temperature is low enough that Gamma_0 selects the basin
    X, Y = O.centre(x, a), O.centre(y, b)
    found = np.inf
    for s in range(12):
        g0 = 0.5 * np.random.default_rng(100 + s).standard_normal((2, 2))
        res = O.cnt_gw(a, b, X, Y, 0.05, 1e-4, 30, 200, gamma0=g0)
        found = min(found, O.quartic_loss(cx, cy, res.pi))
    assert found >= best * (1 - 1e-9)
    assert found - best <= 1e-9 * best


def test_rigid_motion_invariance():
    rng = np.random.default_rng(14)
    n, m = 9, 8
    x = rng.standard_normal((n, 3))
    y = rng.standard_normal((m, 3))
    a = rng.dirichlet(np.ones(n) * 2)
    b = rng.dirichlet(np.ones(m) * 2)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    y2 = y @ q.T + np.array([0.3, -2.0, 1.1])
    out = []
    for yy in (y, y2):
        X, Y = O.centre(x, a), O.centre(yy, b)
        res = O.cnt_gw(a, b, X, Y, 0.1, 0.1, 6, 200)
        out.append((O.lifted_loss(X, Y, a, b, res.pi), res.pi))
    assert abs(out[0][0] - out[1][0]) <= 1e-10 * abs(out[0][0])
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-12


def test_isometric_inputs_reach_zero():
    rng = np.random.default_rng(15)
    n = 8
    x = rng.uniform(-1, 1, (n, 2))
    q, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    perm = rng.permutation(n)
    y = x[perm] @ q.T + 0.5
    a = np.full(n, 1 / n)
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    X, Y = O.centre(x, a), O.centre(y, a)
    losses = []
    for eps_end in (1e-2, 1e-3):
        best = np.inf
        for s in range(6):
            g0 = np.random.default_rng(200 + s).standard_normal((2, 2))
            res = O.cnt_gw(a, a, X, Y, 1.0, eps_end, 40, 400, gamma0=g0)
            best = min(best, O.quartic_loss(cx, cy, res.pi))
        losses.append(best)
    scale = O.quartic_loss(cx, cy, np.outer(a, a))
    assert losses[1] < losses[0]
    assert losses[1] < 1e-4 * scale


def test_monotone_objective_and_dual_descent_bound():
    rng = np.random.default_rng(16)
    n, m = 8, 7
    x = rng.standard_normal((n, 2))
    y = rng.standard_normal((m, 2)) * 1.2
    a = rng.dirichlet(np.ones(n) * 2)
    b = rng.dirichlet(np.ones(m) * 2)
    X, Y = O.centre(x, a), O.centre(y, b)
    eps = 0.15
    g0 = rng.standard_normal((2, 2))
    res = O.cnt_gw(a, b, X, Y, eps, eps, 12, 0, gamma0=g0, record=True, inner_tol=1e-14)
    objs = [O.egw_objective(X, Y, a, b, h["pi"], eps) for h in res.history]
    assert all(objs[k + 1] <= objs[k] + 1e-11 for k in range(len(objs) - 1))
    gammas = [g0] + [h["gamma"] for h in res.history]
    steps = sum(float(np.sum((gammas[k] - gammas[k + 1]) ** 2)) for k in range(len(gammas) - 1))
    drop = O.dual_function(X, Y, a, b, gammas[0], eps) - O.dual_function(X, Y, a, b, gammas[-1], eps)
    assert steps <= drop + 1e-10


def test_dual_descent_step_is_half_gradient():
    """Proposition 4.4: Gamma_{t+1} = Gamma_t - grad Phi_eps(Gamma_t) / 2;
    check grad Phi by central differences of Phi."""
    rng = np.random.default_rng(17)
    n, m = 6, 5
    X = O.centre(rng.standard_normal((n, 2)), np.full(n, 1 / n))
    Y = O.centre(rng.standard_normal((m, 2)), np.full(m, 1 / m))
    a = np.full(n, 1 / n)
    b = np.full(m, 1 / m)
    eps = 0.5
    g0 = rng.standard_normal((2, 2))
    res = O.cnt_gw(a, b, X, Y, eps, eps, 1, 6000, gamma0=g0)
    h = 1e-5
    grad = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            e = np.zeros((2, 2))
            e[i, j] = h
            grad[i, j] = (O.dual_function(X, Y, a, b, g0 + e, eps)
                          - O.dual_function(X, Y, a, b, g0 - e, eps)) / (2 * h)
    assert np.abs(res.gamma - (g0 - 0.5 * grad)).max() < 1e-7


def test_large_temperature_limit():
    rng = np.random.default_rng(18)
    x = rng.standard_normal((7, 2))
    y = rng.standard_normal((6, 2))
    a = rng.dirichlet(np.ones(7))
    b = rng.dirichlet(np.ones(6))
    X, Y = O.centre(x, a), O.centre(y, b)
    res = O.cnt_gw(a, b, X, Y, 1e5, 1e5, 3, 50)
    assert np.abs(res.pi / np.outer(a, b) - 1).max() < 1e-3
    assert np.abs(res.gamma).max() < 1e-3 * np.abs(X).max() * np.abs(Y).max()


def test_schedule_is_geometric():
    s = O.eps_schedule(0.1, 0.005, 30)
    assert s[0] == 0.1 and abs(s[-1] - 0.005) < 1e-15
    ratios = s[1:] / s[:-1]
    assert np.abs(ratios - ratios[0]).max() < 1e-12
    assert np.all(O.eps_schedule(0.01, 0.01, 20) == 0.01)
