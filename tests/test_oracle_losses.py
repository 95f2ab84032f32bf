"""Pins of the oracle's loss evaluators against the GW definition itself.

P1: the lifted form of Lemma C.1 equals the quartic GW loss (Eq. GW_loss)
    for every exactly feasible coupling.
P2: the constant C(alpha, beta) of Lemma C.1 against its moment closed form,
    including the paper's statement C(alpha, alpha) = 8 |Sigma|^2 + 4 int |x|^4.
"""
import itertools

import numpy as np
import pytest

from oracle import gw_oracle as O


def _pair(seed, n, m, dx, dy, dirichlet=True):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, dx))
    y = 0.7 * rng.standard_normal((m, dy)) + 0.3
    if dirichlet:
        a = rng.dirichlet(np.ones(n) * 2)
        b = rng.dirichlet(np.ones(m) * 2)
    else:
        a = np.full(n, 1.0 / n)
        b = np.full(m, 1.0 / m)
    return rng, x, a, y, b


def _feasible_plans(rng, a, b):
    """Exactly feasible couplings: product plan and a Sinkhorn-projected
    random plan (marginals to 1e-15)."""
    yield np.outer(a, b)
    c = rng.standard_normal((len(a), len(b)))
    f, g = O.sinkhorn_converged(a, b, c, 0.7, tol=1e-15)
    yield O.plan(a, b, f, g, c, 0.7)


@pytest.mark.parametrize("seed,n,m,dx,dy", [(0, 5, 6, 2, 2), (1, 7, 4, 3, 2), (2, 6, 6, 1, 3)])
def test_lifted_equals_quartic_literal(seed, n, m, dx, dy):
    rng, x, a, y, b = _pair(seed, n, m, dx, dy)
    X, Y = O.centre(x, a), O.centre(y, b)
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)       # raw points: GW only sees distances
    for pi in _feasible_plans(rng, a, b):
        assert O.marginal_error(pi, a, b) < 1e-14
        lit = O.quartic_loss_literal(cx, cy, pi)
        lif = O.lifted_loss(X, Y, a, b, pi)
        assert abs(lit - lif) <= 1e-11 * max(1.0, abs(lit))
        assert abs(O.quartic_loss(cx, cy, pi) - lit) <= 1e-11 * max(1.0, abs(lit))


def test_lifted_equals_quartic_permutation():
    rng, x, a, y, b = _pair(3, 6, 6, 2, 2, dirichlet=False)
    X, Y = O.centre(x, a), O.centre(y, b)
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    for perm in list(itertools.permutations(range(6)))[::37]:
        pi = np.zeros((6, 6))
        pi[np.arange(6), perm] = 1.0 / 6
        lit = O.quartic_loss_literal(cx, cy, pi)
        assert abs(O.lifted_loss(X, Y, a, b, pi) - lit) <= 1e-11 * max(1.0, lit)


def test_quartic_rearrangement_any_plan():
    """The exact rearrangement must also hold for infeasible plans."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((5, 2))
    y = rng.standard_normal((4, 2))
    pi = rng.uniform(size=(5, 4))
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    lit = O.quartic_loss_literal(cx, cy, pi)
    assert abs(O.quartic_loss(cx, cy, pi) - lit) <= 1e-11 * lit


def test_lifted_differs_when_infeasible():
    """Lemma C.1 uses the marginals: an infeasible plan breaks the identity
    (guards against an evaluator that silently renormalises)."""
    rng, x, a, y, b = _pair(5, 5, 5, 2, 2)
    X, Y = O.centre(x, a), O.centre(y, b)
    pi = np.outer(a, b) * 1.3
    cx, cy = O.sqdist(x, x), O.sqdist(y, y)
    assert abs(O.lifted_loss(X, Y, a, b, pi) - O.quartic_loss(cx, cy, pi)) > 1e-3


def _moments(X, w):
    n2 = np.sum(X * X, 1)
    sig = (w[:, None] * X).T @ X
    return float(w @ n2), float(w @ (n2 * n2)), float(np.sum(sig * sig))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_constant_closed_form(seed):
    """For centred measures, int int |x - x'|^4 = 2 m4 + 4 |Sigma|^2 + 2 s^2
    (expand |x - x'|^4 and drop the odd moments), so
    C = that for x + that for y - 4 s_x s_y."""
    rng, x, a, y, b = _pair(seed, 9, 7, 3, 2)
    X, Y = O.centre(x, a), O.centre(y, b)
    sx, m4x, sigx = _moments(X, a)
    sy, m4y, sigy = _moments(Y, b)
    closed = (2 * m4x + 4 * sigx + 2 * sx * sx) + (2 * m4y + 4 * sigy + 2 * sy * sy) - 4 * sx * sy
    assert abs(O.constant_c(X, Y, a, b) - closed) <= 1e-12 * abs(closed)


def test_constant_self_paper_statement():
    """Appendix C states C(alpha, alpha) = 8 |Sigma_alpha|^2 + 4 int |x|^4."""
    rng, x, a, _, _ = _pair(7, 11, 3, 3, 3)
    X = O.centre(x, a)
    _, m4, sig = _moments(X, a)
    assert abs(O.constant_c(X, X, a, a) - (8 * sig + 4 * m4)) <= 1e-12 * (8 * sig + 4 * m4)


def test_kl_and_marginal_error_definitions():
    a = np.array([0.25, 0.75])
    b = np.array([0.5, 0.5])
    pi = np.array([[0.25, 0.0], [0.25, 0.5]])
    # KL = 0.25 log 2 + 0.25 log(0.25/0.375) + 0.5 log(0.5/0.375)
    want = 0.25 * np.log(2) + 0.25 * np.log(0.25 / 0.375) + 0.5 * np.log(0.5 / 0.375)
    assert abs(O.kl_divergence(pi, a, b) - want) < 1e-15
    assert O.marginal_error(pi, a, b) == 0.0
    assert abs(O.marginal_error(pi * 2, a, b) - 2.0) < 1e-15
