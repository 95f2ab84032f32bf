"""Gradients at the full size of the differentiation workload: 50,000 x
30,000 points in d = 16, Dirichlet(1) weights, |x - x'| lifted to D = 64
(2048 landmarks, frozen after the first lift), FP32.

The envelope gradient is the derivative of the converged objective.  At the
workload's eps = 0.01 its 20 x 50 schedule ends far from a feasible coupling
(marginal error ~3e-2, and still ~2e-2 after 3000 more iterations), so the
finite-difference check runs at eps = 0.05, where the same schedule plus a
polish converges; the oracle's gradient is compared on small inputs in
test_gpu_grad.py, including a subsample of this workload.

Property checks that hold at any size: central differences of the polished
EGW objective, each solve warm-started from the polished state, against the
analytic directional derivative.  Directions: the gradient itself (h =
1e-3) and random moves of O(h) per point and simplex-tangent weight moves
that keep the weights positive (h = 1e-2: at 1e-3 their objective changes
are ~1e-5 of its value, where the FP32 solve's ~3e-7 relative floor would
dominate; the O(h^2) truncation stays below 1e-3).
"""
import numpy as np
import pytest
import torch

from workloads import config5_grad, landmark_indices

pytestmark = pytest.mark.gpu

H_GRAD, H_RAND = 1e-3, 1e-2
EPS = 0.05


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def test_c5_gradients_against_finite_differences(gw):
    prob = config5_grad()
    x, a, y, b = dev(prob.x), dev(prob.a / prob.a.sum()), dev(prob.y), dev(prob.b / prob.b.sum())
    ctx = gw.Context()
    for side, (n, seed) in enumerate(((prob.n, 5101), (prob.m, 5102))):
        ctx.set_penalty(side, "power", p=1.0, lifted_dim=64, n_landmarks=2048)
        ctx.set_landmarks(side, landmark_indices(n, 2048, seed))
    eps = EPS
    base = ctx.solve(x, a, y, b, eps, eps, prob.n_outer, prob.n_inner)
    pol = ctx.loss_and_grad(x, a, y, b, eps, eps, 10, 300, gamma0=base["gamma"], f0=base["f"], g0=base["g"])
    print(f"C5: schedule Err {base['marginal_err']:.2e}, polished Err {pol['marginal_err']:.2e}, "
          f"loss {pol['egw_objective']:.8g}")
    state = dict(gamma0=pol["gamma"], f0=pol["f"], g0=pol["g"])

    def objective(xx, aa):
        return ctx.solve(xx, aa, y, b, eps, eps, 4, 300, **state)["egw_objective"]

    gx, ga = pol["grad_x"], pol["grad_a"]
    rng = np.random.default_rng(5103)
    dirs = [gx / gx.abs().max()] + [dev(rng.standard_normal(prob.x.shape)) for _ in range(3)]
    worst = 0.0
    for k, d in enumerate(dirs):
        h = H_GRAD if k == 0 else H_RAND
        fd = (objective(x + h * d, a) - objective(x - h * d, a)) / (2 * h)
        an = float((gx.double() * d.double()).sum())
        rel = abs(fd - an) / abs(an)
        worst = max(worst, rel)
        print(f"  position direction {k}: fd {fd:.6e} analytic {an:.6e} rel {rel:.2e}")
    for k in range(2):
        u = rng.standard_normal(prob.n)
        da = prob.a * (u - prob.a @ u)
        da = dev(da / np.abs(da / prob.a).max())     # relative change of each weight <= 1
        fd = (objective(x, a + H_RAND * da) - objective(x, a - H_RAND * da)) / (2 * H_RAND)
        an = float((ga.double() * da.double()).sum())
        rel = abs(fd - an) / abs(an)
        worst = max(worst, rel)
        print(f"  weight direction {k}: fd {fd:.6e} analytic {an:.6e} rel {rel:.2e}")
    assert pol["marginal_err"] < 1e-4
    assert worst < 2e-2
