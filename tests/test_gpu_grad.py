"""GPU envelope gradients (gw_loss_and_grad through the C ABI) against the
FP64 oracle's gradients of a converged solve (Appendix B.6).

The expected values come from tests/golden/make_grad_golden.py (oracle
only): the converged Gamma* and potentials f*, g* of Algorithm 1 and the
gradients there, for
seeded inputs from workloads.grad_points:

* positions: the oracle's lifted-form gradient (its pins tie it to the
  quartic envelope and to finite differences), chained through centring and,
  for |x - x'|, the frozen Nystrom map;
* weights: the oracle's brute-force potential of the full linearised cost,
  solved to convergence (the GPU uses the lifted form with separable terms).

GW's outer iteration converges slowly, so the GPU starts from the oracle's
converged state (Gamma*, f*, g*) and runs a few iterations there (per-step
parity from the oracle's state); the weight identity needs a feasible
coupling, which the GPU keeps to its FP32 marginal-error floor.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import gw_oracle as O
from workloads import c5_subsample, grad_points

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def _rel(u, v):
    return float(np.abs(u - v).max() / np.abs(v).max())


def _case(name):
    with open(os.path.join(GOLD, f"grad_{name}.json")) as fh:
        gold = json.load(fh)
    if gold.get("inputs") == "c5_subsample":
        x, a, y, b = c5_subsample(gold["n"], gold["m"], gold["seed"])
    else:
        noise = 0.02 if gold["penalty"] == "power" else 0.05
        x, a, y, b = grad_points(gold["seed"], gold["n"], gold["m"], gold["d"], noise=noise,
                                 scale=gold.get("scale", 1.0))
    return gold, x, a, y, b


def _context(gw, gold, x, a, y, b):
    """Context with the case's penalty, and Gamma* in the GPU's feature
    basis: landmark eigenvectors carry a sign per coordinate, matched here
    against the oracle's features of the same landmarks."""
    ctx = gw.Context()
    gam = np.array(gold["gamma"])
    if gold["penalty"] != "power":
        ctx.set_penalty(2, gold["penalty"])
        return ctx, gam
    D, nl = gold["lifted_dim"], gold["n_landmarks"]
    signs = []
    for side, (pts, w, key) in enumerate(((x, a, "landmarks_x"), (y, b, "landmarks_y"))):
        idx = np.array(gold[key])
        ctx.set_penalty(side, "power", p=1.0, lifted_dim=D, n_landmarks=nl)
        ctx.set_landmarks(side, idx)
        Fg = ctx.lift(side, dev(pts), dev(w)).cpu().numpy().astype(np.float64)
        Fo = O.landmark_features(pts, w, O.fit_landmarks(pts[idx], 1.0, D))
        s = np.sign(np.sum(Fg * Fo, axis=0))
        assert np.abs(Fg * s - Fo).max() < 1e-4 * np.abs(Fo).max()
        signs.append(s)
    return ctx, signs[0][:, None] * gam * signs[1][None, :]


@pytest.mark.parametrize("case,prec,tol", [
    ("sqeuclid", "fp32", 1e-4),
    ("features40", "fp32", 1e-4),
    ("features40", "bf16x3", 1e-4),
    ("features40", "bf16", 3e-2),
    ("power16", "fp32", 1e-4),
    ("c5sub", "fp32", 1e-4),
    ("c5sub", "bf16", 3e-2),
])
def test_gradients_match_oracle(gw, case, prec, tol):
    gold, x, a, y, b = _case(case)
    ctx, gam0 = _context(gw, gold, x, a, y, b)
    eps = gold["eps"]
    out = ctx.loss_and_grad(dev(x), dev(a), dev(y), dev(b), eps, eps, 2, 60, precision=prec, gamma0=dev(gam0),
                            f0=dev(gold["f"]), g0=dev(gold["g"]))
    got = {k: out["grad_" + k].cpu().numpy().astype(np.float64) for k in "xayb"}
    errs = {k: _rel(got[k], np.array(gold["grad_" + k])) for k in "xayb"}
    rel_loss = abs(out["egw_objective"] - gold["egw_objective"]) / abs(gold["egw_objective"])
    print(case, prec, "grad rel err", {k: f"{v:.2e}" for k, v in errs.items()}, f"loss rel {rel_loss:.2e}",
          f"GPU Err {out['marginal_err']:.2e}", f"centring {float(a @ got['a']):.2e} {float(b @ got['b']):.2e}")
    assert max(errs.values()) < tol
    # weight gradients are tangent to the simplex
    assert abs(float(a @ got["a"])) < 1e-6 * np.abs(got["a"]).max()
    assert abs(float(b @ got["b"])) < 1e-6 * np.abs(got["b"]).max()


def test_autograd_function(gw):
    """GWLoss through torch.autograd: the value is the ABI's objective and the
    gradients are the ABI's, scaled by the incoming gradient."""
    x, a, y, b = grad_points(63, 200, 180, 2)
    params = dict(eps_start=0.3, eps_end=0.3, n_outer=10, n_inner=100)
    ctx = gw.Context()
    ref = ctx.loss_and_grad(dev(x), dev(a), dev(y), dev(b), **params)
    xt = dev(x).requires_grad_(True)
    at = dev(a).requires_grad_(True)
    loss = gw.gw_loss(xt, at, dev(y), dev(b), context=ctx, **params)
    (3.0 * loss).backward()
    assert loss.item() == ref["egw_objective"]
    assert torch.equal(xt.grad, 3.0 * ref["grad_x"])
    assert torch.equal(at.grad, 3.0 * ref["grad_a"])
