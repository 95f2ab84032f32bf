"""Pins of the oracle's final-step Sinkhorn annealing (Appendix B.1,
"Sinkhorn Annealing": eps_n = eps_0 / sqrt(n) in the last outer step).

* With the square-root decay the plans of the annealed iteration approach
  the unregularised optimal transport plan of that step's cost (Chizat
  2024): on 5 x 5 uniform problems the annealed plan is the optimal
  permutation found by enumerating all 120 permutations, while the plan at
  the starting eps is spread out.
* Only the last outer step is annealed: the earlier steps are those of the
  plain schedule, and the returned eps is eps_T / sqrt(n_inner).
"""
import itertools

import numpy as np
import pytest

from oracle import gw_oracle as O


def _problem(seed, n=5, d=2):
    rng = np.random.default_rng(seed)
    a = np.full(n, 1.0 / n)
    X = O.centre(rng.standard_normal((n, d)), a)
    Y = O.centre(rng.standard_normal((n, d)), a)
    gamma0 = 0.5 * rng.standard_normal((d, d))
    return a, X, Y, gamma0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_annealed_plan_is_the_optimal_permutation(seed):
    a, X, Y, gamma0 = _problem(seed)
    eps = 0.5
    res = O.cnt_gw(a, a, X, Y, eps, eps, 1, 4000, gamma0=gamma0, anneal_final=True)
    # the step's cost, from the oracle's own lift
    zbar = np.concatenate([Y @ gamma0.T, 0.5 * np.sum(Y * Y, 1, keepdims=True)], axis=1)
    cbar = O.sqdist(O.lift(X), zbar)
    n = len(a)
    best = min(itertools.permutations(range(n)), key=lambda p: sum(cbar[i, p[i]] for i in range(n)))
    target = np.zeros((n, n))
    target[np.arange(n), best] = 1.0 / n
    plain = O.cnt_gw(a, a, X, Y, eps, eps, 1, 4000, gamma0=gamma0)
    print(seed, np.abs(res.pi - target).max(), np.abs(plain.pi - target).max())
    assert abs(res.eps - eps / np.sqrt(4000)) < 1e-15
    assert np.abs(res.pi - target).max() < 2e-3
    assert np.abs(plain.pi - target).max() > 2e-2


def test_only_the_last_step_is_annealed():
    a, X, Y, _ = _problem(7, n=8, d=3)
    b = np.full(8, 1.0 / 8)
    plain = O.cnt_gw(a, b, X, Y, 0.2, 0.1, 3, 40, record=True)
    ann = O.cnt_gw(a, b, X, Y, 0.2, 0.1, 3, 40, record=True, anneal_final=True)
    for t in range(2):
        assert np.array_equal(plain.history[t]["gamma"], ann.history[t]["gamma"])
    assert np.abs(plain.history[2]["gamma"] - ann.history[2]["gamma"]).max() > 1e-6
    assert ann.eps == pytest.approx(0.1 / np.sqrt(40), rel=1e-15)
    assert plain.eps == pytest.approx(0.1, rel=1e-15)
