"""Position and weight gradients of the Sinkhorn-GW divergence on the GPU
(gw_sgw_grad through the C ABI) against the oracle's envelope gradients at
converged solves (eps = 2, one attractor per problem), and the position
gradient's zero at isometric measures.  The GPU runs 40 x 400 FP32 iterations, converged to the FP32
floor, so the gradients agree to 1e-4 of their largest entry; between
isometric measures the divergence's gradient is below 1e-3 of the pair's
own envelope gradient."""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as O

pytestmark = pytest.mark.gpu
EPS = 2.0


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def _measure(rng, n, d):
    x = f32(rng.standard_normal((n, d)) * np.array([1.0, 0.6, 0.3][:d]))
    a = f32(rng.dirichlet(np.ones(n) * 3))
    return x, a / a.sum()


def test_sgw_gradient_matches_oracle(gw):
    rng = np.random.default_rng(50)
    x, a = _measure(rng, 40, 2)
    y, b = _measure(rng, 35, 2)
    print("sgw grad n=40 m=35", flush=True)
    res = gw.Context().sgw_grad(dev(x), dev(a), dev(y), dev(b), EPS, EPS, 40, 400)
    gx_ref, gy_ref = O.sgw_grad_positions(a, b, x, y, EPS)
    gx, gy = res["grad_x"].cpu().numpy(), res["grad_y"].cpu().numpy()
    ex = np.abs(gx - gx_ref).max() / np.abs(gx_ref).max()
    ey = np.abs(gy - gy_ref).max() / np.abs(gy_ref).max()
    print("errors", ex, ey, "sgw", res["sgw"], "err", res["marginal_err"])
    assert ex <= 1e-4 and ey <= 1e-4


def test_sgw_gradient_vanishes_between_isometric_measures(gw):
    rng = np.random.default_rng(51)
    x, a = _measure(rng, 50, 2)
    th = 1.1
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    perm = rng.permutation(50)
    y = f32((x @ R.T + np.array([2.0, -0.5]))[perm])
    b = a[perm]
    ctx = gw.Context()
    res = ctx.sgw_grad(dev(x), dev(a), dev(y), dev(b), EPS, EPS, 40, 400)
    pair = ctx.loss_and_grad(dev(x), dev(a), dev(y), dev(b), EPS, EPS, 40, 400, want=("x",))
    scale = pair["grad_x"].abs().max().item()
    print("isometric: |grad| max", res["grad_x"].abs().max().item(), res["grad_y"].abs().max().item(), "scale", scale)
    assert scale > 1e-2
    assert res["grad_x"].abs().max().item() <= 1e-3 * scale
    assert res["grad_y"].abs().max().item() <= 1e-3 * scale


def test_lifted_sgw_gradient_matches_oracle(gw):
    # |x - x'| lifted to D = 4 by landmark kernel PCA on the first points of
    # each measure (the same indices on both sides of the comparison; the
    # eigenvectors' signs may differ, which leaves the objective and the
    # position gradients unchanged)
    rng = np.random.default_rng(53)
    x, a = _measure(rng, 40, 2)
    y, b = _measure(rng, 35, 2)
    ix, iy = np.arange(30), np.arange(28)
    ctx = gw.Context()
    for side, idx in ((0, ix), (1, iy)):
        ctx.set_penalty(side, "power", p=1.0, lifted_dim=4, n_landmarks=len(idx))
        ctx.set_landmarks(side, idx)
    print("lifted sgw grad n=40 m=35 D=4", flush=True)
    res = ctx.sgw_grad(dev(x), dev(a), dev(y), dev(b), EPS, EPS, 40, 400)
    lmx, lmy = O.fit_landmarks(x[ix], 1.0, 4), O.fit_landmarks(y[iy], 1.0, 4)
    gx_ref, gy_ref = O.sgw_grad_positions_lifted(a, b, x, y, EPS, lmx, lmy)
    gx, gy = res["grad_x"].cpu().numpy(), res["grad_y"].cpu().numpy()
    ex = np.abs(gx - gx_ref).max() / np.abs(gx_ref).max()
    ey = np.abs(gy - gy_ref).max() / np.abs(gy_ref).max()
    ref_val = O.sgw_value_converged_lifted(a, b, x, y, EPS, lmx, lmy)
    print("lifted errors", ex, ey, "sgw", res["sgw"], "oracle", ref_val, "err", res["marginal_err"])
    assert ex <= 1e-4 and ey <= 1e-4
    assert abs(res["sgw"] - ref_val) <= 1e-4 * abs(res["gw_xy"])


def test_sgw_weight_gradients_match_oracle(gw):
    # 9 and 8 points (the oracle's converged solves of larger clouds at
    # eps = 2 are slow to reach the FP64 floor); weight gradients centred
    # along the simplex on both sides
    rng = np.random.default_rng(42)
    x, a = _measure(rng, 9, 2)
    y, b = _measure(rng, 8, 2)
    print("sgw weight gradients n=9 m=8", flush=True)
    res = gw.Context().sgw_grad(dev(x), dev(a), dev(y), dev(b), EPS, EPS, 40, 400, weights=True)
    ga_ref, gb_ref = O.sgw_grad_weights(a, b, x, y, EPS, tol=1e-11)
    ga = res["grad_a"].cpu().numpy().astype(np.float64)
    gb = res["grad_b"].cpu().numpy().astype(np.float64)
    ea = np.abs(ga - ga_ref).max() / np.abs(ga_ref).max()
    eb = np.abs(gb - gb_ref).max() / np.abs(gb_ref).max()
    print("weight errors", ea, eb, "err", res["marginal_err"])
    assert abs(a @ ga) <= 1e-5 * np.abs(ga).max() and abs(b @ gb) <= 1e-5 * np.abs(gb).max()
    assert ea <= 1e-4 and eb <= 1e-4


def test_lifted_sgw_weight_gradients_match_oracle(gw):
    rng = np.random.default_rng(53)
    x, a = _measure(rng, 40, 2)
    y, b = _measure(rng, 35, 2)
    ix, iy = np.arange(30), np.arange(28)
    ctx = gw.Context()
    for side, idx in ((0, ix), (1, iy)):
        ctx.set_penalty(side, "power", p=1.0, lifted_dim=4, n_landmarks=len(idx))
        ctx.set_landmarks(side, idx)
    print("lifted sgw weight gradients n=40 m=35 D=4", flush=True)
    res = ctx.sgw_grad(dev(x), dev(a), dev(y), dev(b), EPS, EPS, 40, 400, weights=True)
    lmx, lmy = O.fit_landmarks(x[ix], 1.0, 4), O.fit_landmarks(y[iy], 1.0, 4)
    ga_ref, gb_ref = O.sgw_grad_weights_lifted(a, b, x, y, EPS, lmx, lmy)
    ga = res["grad_a"].cpu().numpy().astype(np.float64)
    gb = res["grad_b"].cpu().numpy().astype(np.float64)
    ea = np.abs(ga - ga_ref).max() / np.abs(ga_ref).max()
    eb = np.abs(gb - gb_ref).max() / np.abs(gb_ref).max()
    print("lifted weight errors", ea, eb, "err", res["marginal_err"])
    assert ea <= 1e-4 and eb <= 1e-4
