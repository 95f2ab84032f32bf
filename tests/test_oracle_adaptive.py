"""Pins of Algorithm 6's adaptive Sinkhorn counts in the oracle's CNT-GW
(Appendix B, "Adaptive Sinkhorn Iterations").

* With converged inner solves the EGW objective decreases at every outer
  step (Theorem 4.5), so the rule never fires and the run equals the fixed
  one.
* From a count too small to converge (one iteration), the rule fires and the
  run ends at an EGW local minimum, as the paper guarantees: a coupling with
  exact marginals, from which the exact algorithm (Sinkhorn solved to
  convergence at every step) does not move.  The fixed one-iteration run
  ends far from a coupling."""
import numpy as np

from oracle import gw_oracle as O


def _problem(seed=5, n=60, m=50):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 2)) * np.array([1.0, 0.5])
    y = rng.standard_normal((m, 2)) * np.array([0.9, 0.6])
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    return a, b, O.centre(x, a), O.centre(y, b)


def test_converged_inner_solves_never_double():
    a, b, X, Y = _problem()
    fixed = O.cnt_gw(a, b, X, Y, 0.3, 0.3, 12, 2000)
    adapt = O.cnt_gw(a, b, X, Y, 0.3, 0.3, 12, 2000, adaptive=True)
    assert adapt.doublings == 0 and adapt.n_inner_final == 2000
    assert np.array_equal(adapt.gamma, fixed.gamma)


def test_too_few_iterations_double_and_reach_a_local_minimum():
    a, b, X, Y = _problem()
    eps = 0.3
    fixed = O.cnt_gw(a, b, X, Y, eps, eps, 150, 1)
    adapt = O.cnt_gw(a, b, X, Y, eps, eps, 150, 1, adaptive=True)
    assert adapt.doublings >= 1 and adapt.n_inner_final == 2 ** adapt.doublings
    assert O.marginal_error(adapt.pi, a, b) < 1e-10
    assert O.marginal_error(fixed.pi, a, b) > 1e-2
    gamma, pi, _, _ = O.cnt_gw_converged(a, b, X, Y, eps, gamma0=adapt.gamma, tol=1e-12)
    assert np.max(np.abs(gamma - adapt.gamma)) < 1e-8
    e_ad = O.egw_objective(X, Y, a, b, adapt.pi, eps)
    assert abs(O.egw_objective(X, Y, a, b, pi, eps) - e_ad) < 1e-9 * abs(e_ad)
