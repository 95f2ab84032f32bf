"""Pins of the oracle's C Sinkhorn loop (oracle/sinkhorn.c), used for the
large golden problems.  It is pinned like the NumPy loop, by what fixes the
EOT solution independently of either: the textbook matrix-scaling routine
at convergence, the closed forms for separable costs and a single source
point, one step against the operators written out as explicit sums; and it
must equal the NumPy loop to float64 rounding."""
import numpy as np
import pytest

from oracle import gw_oracle as O


def _scaling(a, b, c, eps, n_iter=20000):
    k = np.exp(-c / eps)
    v = np.ones(len(b))
    for _ in range(n_iter):
        u = a / (k @ v)
        v = b / (k.T @ u)
    return u[:, None] * k * v[None, :]


@pytest.mark.parametrize("symmetric", [True, False])
def test_converges_to_textbook_scaling(symmetric):
    rng = np.random.default_rng(10)
    a = rng.dirichlet(np.ones(9))
    b = rng.dirichlet(np.ones(7))
    c = rng.uniform(0, 1, (9, 7))
    eps = 0.2
    f, g = O.sinkhorn(a, b, c, eps, 3000, symmetric=symmetric, backend="c")
    assert np.abs(O.plan(a, b, f, g, c, eps) - _scaling(a, b, c, eps)).max() < 1e-13


@pytest.mark.parametrize("symmetric", [True, False])
def test_one_step_equals_explicit_operators(symmetric):
    rng = np.random.default_rng(11)
    a = rng.dirichlet(np.ones(4))
    b = rng.dirichlet(np.ones(3))
    c = rng.standard_normal((4, 3))
    f0, g0 = rng.standard_normal(4), rng.standard_normal(3)
    eps = 0.5
    f1, g1 = O.sinkhorn(a, b, c, eps, 1, f0, g0, symmetric=symmetric, backend="c")
    tf = np.array([-eps * np.log(sum(b[j] * np.exp((g0[j] - c[i, j]) / eps) for j in range(3))) for i in range(4)])
    fg = f0 if symmetric else tf
    tg = np.array([-eps * np.log(sum(a[i] * np.exp((fg[i] - c[i, j]) / eps) for i in range(4))) for j in range(3)])
    if symmetric:
        tf, tg = 0.5 * (f0 + tf), 0.5 * (g0 + tg)
    assert np.abs(f1 - tf).max() < 1e-14 and np.abs(g1 - tg).max() < 1e-14


def test_separable_cost_and_single_point():
    rng = np.random.default_rng(12)
    a = rng.dirichlet(np.ones(5))
    b = rng.dirichlet(np.ones(4))
    c = rng.standard_normal(5)[:, None] + rng.standard_normal(4)[None, :]
    f, g = O.sinkhorn(a, b, c, 0.05, 200, backend="c")
    assert np.abs(O.plan(a, b, f, g, c, 0.05) - np.outer(a, b)).max() < 1e-14
    c1 = rng.standard_normal((1, 4))
    f, g = O.sinkhorn(np.ones(1), b, c1, 0.01, 500, symmetric=False, backend="c")
    assert np.abs(O.plan(np.ones(1), b, f, g, c1, 0.01)[0] - b).max() < 1e-13


@pytest.mark.parametrize("symmetric", [True, False])
def test_equals_numpy_loop(symmetric):
    """Tiny temperature (the max shift matters), ragged sizes, non-uniform
    weights: 40 iterations agree with the NumPy loop to float64 rounding."""
    rng = np.random.default_rng(13)
    n, m = 301, 157
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    c = rng.uniform(0.0, 3.0, (n, m))
    eps = 2e-3
    f0, g0 = 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(m)
    fn, gn = O.sinkhorn(a, b, c, eps, 40, f0, g0, symmetric)
    fc, gc = O.sinkhorn(a, b, c, eps, 40, f0, g0, symmetric, backend="c")
    assert np.abs(fn - fc).max() < 1e-12 and np.abs(gn - gc).max() < 1e-12


def test_cnt_gw_backends_agree():
    rng = np.random.default_rng(14)
    X = O.centre(rng.standard_normal((80, 3)), np.full(80, 1 / 80))
    Y = O.centre(rng.standard_normal((70, 3)), np.full(70, 1 / 70))
    a, b = np.full(80, 1 / 80), np.full(70, 1 / 70)
    r1 = O.cnt_gw(a, b, X, Y, 0.5, 0.05, 6, 30)
    r2 = O.cnt_gw(a, b, X, Y, 0.5, 0.05, 6, 30, backend="c")
    assert np.abs(r1.gamma - r2.gamma).max() < 1e-11
    assert abs(O.lifted_loss(X, Y, a, b, r1.pi) - O.lifted_loss(X, Y, a, b, r2.pi)) < 1e-12
