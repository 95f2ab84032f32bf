"""Pins of the oracle's log-domain Sinkhorn (Algorithms 2 and 3).

P3: the EOT optimum is unique, so a converged run must reproduce the plan of
an independent textbook routine (matrix scaling on the Gibbs kernel), satisfy
the marginals, and have dual value equal to primal value.  Special cases with
known closed-form answers: separable costs give a x b, N = 1 gives pi = b.
"""
import numpy as np
import pytest

from oracle import gw_oracle as O


def _scaling_sinkhorn(a, b, c, eps, n_iter=20000):
    """Textbook matrix scaling: K = exp(-C/eps), u = a / (K v), v = b / (K^T u),
    pi = diag(u) K diag(v).  Independent of the log-domain code."""
    k = np.exp(-c / eps)
    v = np.ones(len(b))
    for _ in range(n_iter):
        u = a / (k @ v)
        v = b / (k.T @ u)
    return u[:, None] * k * v[None, :]


@pytest.mark.parametrize("symmetric", [True, False])
def test_matches_textbook_scaling(symmetric):
    rng = np.random.default_rng(0)
    a = rng.dirichlet(np.ones(8))
    b = rng.dirichlet(np.ones(6))
    c = rng.uniform(0, 1, (8, 6))
    eps = 0.2
    f, g = O.sinkhorn_converged(a, b, c, eps, tol=1e-15, symmetric=symmetric)
    pi = O.plan(a, b, f, g, c, eps)
    ref = _scaling_sinkhorn(a, b, c, eps)
    assert np.abs(pi - ref).max() < 1e-13
    assert O.marginal_error(pi, a, b) < 1e-14


def test_dual_equals_primal():
    """At the optimum <a,f> + <b,g> = <C,pi> + eps KL(pi | a x b)."""
    rng = np.random.default_rng(1)
    a = rng.dirichlet(np.ones(7))
    b = rng.dirichlet(np.ones(9))
    c = rng.standard_normal((7, 9))
    eps = 0.3
    f, g = O.sinkhorn_converged(a, b, c, eps, tol=1e-15)
    pi = O.plan(a, b, f, g, c, eps)
    dual = a @ f + b @ g
    primal = float(np.sum(c * pi)) + eps * O.kl_divergence(pi, a, b)
    assert abs(dual - primal) < 1e-12 * max(1.0, abs(primal))


def test_separable_cost_gives_product_plan():
    rng = np.random.default_rng(2)
    a = rng.dirichlet(np.ones(5))
    b = rng.dirichlet(np.ones(4))
    c = rng.standard_normal(5)[:, None] + rng.standard_normal(4)[None, :]
    f, g = O.sinkhorn(a, b, c, 0.05, 200)
    assert np.abs(O.plan(a, b, f, g, c, 0.05) - np.outer(a, b)).max() < 1e-14


def test_single_source_point():
    rng = np.random.default_rng(3)
    b = rng.dirichlet(np.ones(6))
    c = rng.standard_normal((1, 6))
    f, g = O.sinkhorn_converged(np.ones(1), b, c, 0.01, tol=1e-14)
    assert np.abs(O.plan(np.ones(1), b, f, g, c, 0.01)[0] - b).max() < 1e-13


def test_symmetric_and_alternating_reach_same_plan():
    rng = np.random.default_rng(4)
    a = rng.dirichlet(np.ones(10))
    b = rng.dirichlet(np.ones(10))
    c = rng.uniform(0, 2, (10, 10))
    eps = 0.1
    f1, g1 = O.sinkhorn_converged(a, b, c, eps, tol=1e-15, symmetric=True)
    f2, g2 = O.sinkhorn_converged(a, b, c, eps, tol=1e-15, symmetric=False)
    assert np.abs(O.plan(a, b, f1, g1, c, eps) - O.plan(a, b, f2, g2, c, eps)).max() < 1e-13


def test_symmetric_step_is_average_of_operators():
    """Algorithm 3 is the average of the identity and the Sinkhorn operator,
    both read at iterate n; Algorithm 2 applies the operators in sequence."""
    rng = np.random.default_rng(5)
    a = rng.dirichlet(np.ones(4))
    b = rng.dirichlet(np.ones(3))
    c = rng.standard_normal((4, 3))
    f0 = rng.standard_normal(4)
    g0 = rng.standard_normal(3)
    eps = 0.5
    f1, g1 = O.sinkhorn(a, b, c, eps, 1, f0, g0, symmetric=True)
    # direct evaluation of the operators by explicit loops
    tf = np.array([-eps * np.log(sum(b[j] * np.exp((g0[j] - c[i, j]) / eps) for j in range(3)))
                   for i in range(4)])
    tg = np.array([-eps * np.log(sum(a[i] * np.exp((f0[i] - c[i, j]) / eps) for i in range(4)))
                   for j in range(3)])
    assert np.abs(f1 - 0.5 * (f0 + tf)).max() < 1e-14
    assert np.abs(g1 - 0.5 * (g0 + tg)).max() < 1e-14
    f2, g2 = O.sinkhorn(a, b, c, eps, 1, f0, g0, symmetric=False)
    tg2 = np.array([-eps * np.log(sum(a[i] * np.exp((tf[i] - c[i, j]) / eps) for i in range(4)))
                    for j in range(3)])
    assert np.abs(f2 - tf).max() < 1e-14 and np.abs(g2 - tg2).max() < 1e-14


def test_log_domain_survives_tiny_temperature():
    """Max-shifted LSE: exp(-C/eps) underflows float64 for eps = 2e-3 and
    C >= 1.42 (exp(-710)); the log-domain iteration must not."""
    rng = np.random.default_rng(6)
    a = np.full(6, 1 / 6)
    b = np.full(6, 1 / 6)
    c = rng.uniform(1.5, 2.5, (6, 6))
    assert np.all(np.exp(-c / 2e-3) == 0.0)
    f, g = O.sinkhorn(a, b, c, 2e-3, 300, symmetric=False)
    pi = O.plan(a, b, f, g, c, 2e-3)
    assert np.all(np.isfinite(pi))
    # the last half-step of Algorithm 2 makes the column marginals exact
    assert np.abs(pi.sum(0) - b).max() < 1e-12
    assert O.marginal_error(pi, a, b) < 0.05
