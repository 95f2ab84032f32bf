"""GPU landmark kernel PCA (|x - x'| penalty) against the FP64 oracle.

Eigenvectors are defined up to sign, so features are compared through
invariants: pairwise squared distances of lifted points, the weighted
centring, and the GW solution (equivariant under orthogonal changes of the
feature basis when Gamma_0 = 0)."""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as O
from workloads import config2_fp32, landmark_indices, subsample

pytestmark = pytest.mark.gpu


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def _lift_both(gw, x, a, p, D, idx):
    ctx = gw.Context()
    ctx.set_penalty(0, "power", p=p, lifted_dim=D, n_landmarks=len(idx))
    ctx.set_landmarks(0, idx)
    Xg = ctx.lift(0, dev(x), dev(a)).cpu().numpy().astype(np.float64)
    lm = O.fit_landmarks(f32(x)[idx], p, D)
    Xo = O.landmark_features(f32(x), a, lm)
    return Xg, Xo, lm


@pytest.mark.parametrize("p,D,nl", [(1.0, 32, 256), (0.5, 16, 128), (1.5, 64, 400)])
def test_lift_distances_match(gw, p, D, nl):
    rng = np.random.default_rng(50)
    x = rng.standard_normal((3001, 3)) * 0.5
    a = rng.dirichlet(np.ones(3001) * 3)
    a = f32(a) / f32(a).sum()
    idx = landmark_indices(3001, nl, 7)
    Xg, Xo, lm = _lift_both(gw, x, a, p, D, idx)
    i = rng.integers(0, 3001, 4000)
    k = rng.integers(0, 3001, 4000)
    dg = ((Xg[i] - Xg[k]) ** 2).sum(1)
    do = ((Xo[i] - Xo[k]) ** 2).sum(1)
    scale = do.max()
    err = np.abs(dg - do).max() / scale
    cen = np.abs(a @ Xg).max()
    print(f"p={p} D={D} nl={nl}: max rel distance error {err:.2e}, centring {cen:.2e}")
    assert err < 2e-5
    assert cen < 1e-6


def test_power_penalty_solve_matches_oracle(gw):
    prob = subsample(config2_fp32(n=20_000), 1500, 1400, seed=2999)
    D = 32
    ix = landmark_indices(prob.n, 300, 21)
    iy = landmark_indices(prob.m, 300, 22)
    ctx = gw.Context()
    ctx.set_penalty(0, "power", p=1.0, lifted_dim=D, n_landmarks=300)
    ctx.set_penalty(1, "power", p=1.0, lifted_dim=D, n_landmarks=300)
    ctx.set_landmarks(0, ix)
    ctx.set_landmarks(1, iy)
    a = f32(prob.a) / f32(prob.a).sum()
    b = f32(prob.b) / f32(prob.b).sum()
    res = ctx.solve(dev(prob.x), dev(a), dev(prob.y), dev(b), 0.1, 0.02, 6, 60, precision="fp32")
    X = O.landmark_features(f32(prob.x), a, O.fit_landmarks(f32(prob.x)[ix], 1.0, D))
    Y = O.landmark_features(f32(prob.y), b, O.fit_landmarks(f32(prob.y)[iy], 1.0, D))
    ref = O.cnt_gw(a, b, X, Y, 0.1, 0.02, 6, 60)
    ref_loss = O.lifted_loss(X, Y, a, b, ref.pi)
    rel = abs(res["loss_lift"] - ref_loss) / abs(ref_loss)
    sv_g = np.linalg.svd(res["gamma"].cpu().numpy(), compute_uv=False)
    sv_o = np.linalg.svd(ref.gamma, compute_uv=False)
    print(f"power solve: loss {res['loss_lift']:.8g} oracle {ref_loss:.8g} rel {rel:.2e} "
          f"sv rel {np.abs(sv_g - sv_o).max() / sv_o.max():.2e} err {res['marginal_err']:.2e}")
    assert rel < 1e-4
