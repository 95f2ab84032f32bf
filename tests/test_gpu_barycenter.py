"""GW barycentre flow on the GPU (gw_sgw_barycenter through the C ABI)
against the oracle's flow with converged solves: three descent steps of
(1 - lam) SGW(gamma_z, alpha) + lam SGW(gamma_z, beta) at eps = 2.  The GPU
solves run 40 x 400 FP32 iterations (converged to the FP32 floor), so the
moved points agree to 1e-4 of their extent and the objectives to 1e-5 of
their value; the objective decreases at every step.  The same with
|x - x'|^1.5 lifted by frozen landmark maps, one per measure."""
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


def test_barycenter_flow_matches_oracle(gw):
    rng = np.random.default_rng(70)
    x = f32(rng.standard_normal((12, 2)) * np.array([1.0, 0.4]))
    y = f32(rng.standard_normal((10, 2)) * np.array([0.5, 0.9]))
    z0 = f32(rng.standard_normal((8, 2)) * 0.7)
    a, b, w = np.full(12, 1.0 / 12), np.full(10, 0.1), np.full(8, 0.125)
    lam, step, steps = 0.3, 0.02, 3
    print("barycentre flow 12/10/8 points, 3 steps", flush=True)
    z, obj = gw.Context().sgw_barycenter(dev(x), dev(a), dev(y), dev(b), dev(z0), dev(w), lam, step, steps,
                                         EPS, EPS, 40, 400)
    z_ref, obj_ref = O.sgw_barycenter(a, b, x, y, z0, w, lam, step, steps, EPS, tol=1e-11)
    z = z.cpu().numpy()
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    print("z err", err, "objectives", obj, obj_ref)
    assert err <= 1e-4
    assert np.allclose(obj, obj_ref, rtol=1e-5, atol=0)
    assert all(obj[i + 1] < obj[i] for i in range(steps))
    assert np.abs(z - z0).max() > 1e-2          # the points moved


def test_lifted_barycenter_flow_matches_oracle(gw):
    # |x - x'|^1.5 lifted to D = 3: z's map fitted on z0 (all its points),
    # alpha's and beta's on their first six points; the oracle's flow with
    # the same frozen maps (sgw_barycenter_lifted)
    rng = np.random.default_rng(71)
    x = f32(rng.standard_normal((12, 2)) * np.array([1.0, 0.4]))
    y = f32(rng.standard_normal((10, 2)) * np.array([0.5, 0.9]))
    z0 = f32(rng.standard_normal((8, 2)) * 0.7)
    a, b, w = np.full(12, 1.0 / 12), np.full(10, 0.1), np.full(8, 0.125)
    lam, step, steps, p = 0.3, 0.02, 3, 1.5
    ctx = gw.Context()
    ctx.set_penalty(0, "power", p=p, lifted_dim=3, n_landmarks=8)
    ctx.set_landmarks(0, np.arange(8))
    ctx.set_penalty(1, "power", p=p, lifted_dim=3, n_landmarks=6)
    ctx.set_landmarks(1, np.arange(6))
    print("lifted barycentre flow 12/10/8 points, 3 steps", flush=True)
    # the outer iteration of the lifted (z, alpha) problem converges slowly
    # (the oracle's Gamma is still 3% off after 40 outer steps, 1e-8 after
    # 200 x 50), and the envelope gradient needs the converged map
    z, obj = ctx.sgw_barycenter(dev(x), dev(a), dev(y), dev(b), dev(z0), dev(w), lam, step, steps,
                                EPS, EPS, 200, 50)
    lmz, lma, lmb = O.fit_landmarks(z0, p, 3), O.fit_landmarks(x[:6], p, 3), O.fit_landmarks(y[:6], p, 3)
    z_ref, obj_ref = O.sgw_barycenter_lifted(a, b, x, y, z0, w, lam, step, steps, EPS, lmz, lma, lmb, tol=1e-11)
    z = z.cpu().numpy()
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    print("lifted z err", err, "objectives", obj, obj_ref)
    assert err <= 1e-4
    assert np.allclose(obj, obj_ref, rtol=1e-5, atol=0)
    assert all(obj[i + 1] < obj[i] for i in range(steps))


def test_barycenter_rejects_bad_arguments(gw):
    x = dev(np.random.default_rng(1).standard_normal((6, 2)))
    a = dev(np.full(6, 1.0 / 6))
    ctx = gw.Context()
    with pytest.raises(gw.GWError):
        ctx.sgw_barycenter(x, a, x, a, x, a, 1.5, 0.1, 1, EPS)
    with pytest.raises(gw.GWError):
        ctx.sgw_barycenter(x, a, x, a, x, a, 0.5, -0.1, 1, EPS)
