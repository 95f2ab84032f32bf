"""Multiscale-GW on the GPU (gw_kmeans, gw_interpolate, gw_msgw through the
C ABI) against the oracle's Coarsen, Algorithm 8 and Algorithm 7.

* K-Means: bit-exact.  Both sides decide each assignment with the same
  single-precision operations in the same order, sum the clusters exactly in
  integers and divide once in FP64, so centroids, weights, assignments and
  the cluster count must be identical.
* Interpolate: FP32 against FP64.  The exponent (h - d) / eps' is formed in
  single precision, so each potential carries an error of a few units of
  2^-24 (|h| + |d|): tolerance 2e-6 (1 + max|h| + max|out|).
* Multiscale solve: the loss tolerances of the solver (1e-5 FP32, 1e-3
  BF16) on point clouds whose centring is exact (dyadic coordinates,
  power-of-two sizes, uniform weights), so that both sides cluster the same
  features."""
import math

import numpy as np
import pytest
import torch

from oracle import gw_oracle as O
from workloads import synth

pytestmark = pytest.mark.gpu


def dev(v, dtype=np.float32):
    return torch.tensor(np.asarray(v, dtype=dtype), device="cuda")


def _gmm32(seed, n, d, k=8, sigma=0.08):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1, 1, (k, d))
    x = (means[rng.integers(0, k, n)] + sigma * rng.standard_normal((n, d))).astype(np.float32)
    w = rng.dirichlet(np.ones(n) * 2).astype(np.float32)
    w = (w / w.sum(dtype=np.float64)).astype(np.float32)
    return x, w


def _check_kmeans(gw, X, w, k, n_lloyd, seed):
    ctx = gw.Context()
    print(f"kmeans n={len(X)} D={X.shape[1]} k={k} n_lloyd={n_lloyd} seed={seed}", flush=True)
    res = ctx.kmeans(dev(X), dev(w), k, n_lloyd, seed)
    init = synth.splitmix64_landmarks(len(X), k, seed)
    Xc, wc, assign, kept = O.coarsen(X, w, init, n_lloyd)
    assert res["kc"] == len(kept)
    assert np.array_equal(res["assign"].cpu().numpy().astype(np.int64), assign)
    assert np.array_equal(res["Xc"].cpu().numpy(), Xc)
    assert np.array_equal(res["wc"].cpu().numpy(), wc)
    return res


@pytest.mark.parametrize("n,D,k", [(3000, 3, 301), (2500, 17, 250), (2100, 64, 97), (1000, 100, 40),
                                   (600, 256, 33)])
def test_kmeans_bitexact(gw, n, D, k):
    X, w = _gmm32(100 + D, n, D)
    _check_kmeans(gw, X, w, k, 5, seed=D)


def test_kmeans_edge_cases(gw):
    X, w = _gmm32(7, 513, 5)
    res = _check_kmeans(gw, X, w, 1, 2, seed=1)           # one cluster: the weighted mean
    assert res["kc"] == 1
    res = _check_kmeans(gw, X, w, 513, 3, seed=2)         # one point per cluster: the points themselves
    idx = synth.splitmix64_landmarks(513, 513, 2)
    assert np.array_equal(res["Xc"].cpu().numpy(), X[idx])
    # repeated points: starts that coincide leave clusters empty, and they are dropped
    Xd = np.repeat(X[:40], 8, axis=0)
    wd = np.full(len(Xd), 1.0 / len(Xd), dtype=np.float32)
    res = _check_kmeans(gw, Xd, wd, 120, 4, seed=3)
    assert res["kc"] < 120


@pytest.mark.parametrize("side,D,E", [(0, 3, 2), (1, 3, 2), (0, 32, 32), (1, 64, 48), (0, 130, 7)])
def test_interpolate_matches_oracle(gw, side, D, E):
    rng = np.random.default_rng(10 * side + D)
    nq, nr = 1500, 203
    dq, dr = (D, E) if side == 0 else (E, D)
    P = (rng.standard_normal((nq, dq)) / math.sqrt(dq)).astype(np.float32)
    Q = (rng.standard_normal((nr, dr)) / math.sqrt(dr)).astype(np.float32)
    G = (0.3 * rng.standard_normal((D, E)) / math.sqrt(E)).astype(np.float32)
    w = rng.dirichlet(np.ones(nr)).astype(np.float32)
    h = (0.2 * rng.standard_normal(nr)).astype(np.float32)
    eps = 0.05
    print(f"interpolate side={side} D={D} E={E}", flush=True)
    out = gw.Context().interpolate(side, dev(h), dev(P), dev(Q), dev(w), dev(G), eps).cpu().numpy()
    ref = O.interpolate(h.astype(np.float64), P, Q, w.astype(np.float64), G, eps, side)
    tol = 2e-6 * (1 + np.abs(h).max() + np.abs(ref).max())
    err = np.abs(out - ref).max()
    print("max err", err, "tol", tol)
    assert err <= tol


def _dyadic_cloud(seed, n, d, k=6, sigma=0.08):
    """GMM points on the grid 2^-8, centred exactly (n a power of two), so
    that centring them again leaves every single-precision value unchanged."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1, 1, (k, d)) / math.sqrt(d)
    x = means[rng.integers(0, k, n)] + sigma / math.sqrt(d) * rng.standard_normal((n, d))
    x = np.round(x * 256) / 256
    x = x - x.mean(0)
    assert np.all(x.mean(0) == 0) and np.array_equal(x.astype(np.float32).astype(np.float64), x)
    return x


@pytest.mark.parametrize("prec,d,tol", [("fp32", 3, 1e-5), ("bf16", 16, 1e-3)])
def test_msgw_matches_oracle(gw, prec, d, tol):
    n, m = 1024, 512
    x = _dyadic_cloud(61 + d, n, d)
    y = _dyadic_cloud(62 + d, m, d)
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    coarse = dict(eps_start=0.1, eps_end=0.02, n_outer=10, n_inner=60)
    fine = dict(eps_start=0.02, eps_end=0.02, n_outer=3, n_inner=60)
    rho, n_lloyd, seed = 0.1, 5, 7
    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    print(f"msgw {prec} d={d}", flush=True)
    res = ctx.msgw(dev(x), dev(a), dev(y), dev(b), dict(coarse, precision=prec), dict(fine, precision=prec),
                   rho=rho, n_lloyd=n_lloyd, seed=seed)
    ix = synth.splitmix64_landmarks(n, math.ceil(rho * n), seed)
    iy = synth.splitmix64_landmarks(m, math.ceil(rho * m), seed + 1)
    ref = O.msgw(a, b, x, y, ix, iy, n_lloyd, coarse, fine)
    info = res["info"]
    assert info["n_coarse"] == len(ref.ac) and info["m_coarse"] == len(ref.bc)
    c_loss = O.lifted_loss(ref.Xc, ref.Yc, ref.ac, ref.bc, ref.coarse.pi)
    loss = O.lifted_loss(x, y, a, b, ref.fine.pi)
    egw = O.egw_objective(x, y, a, b, ref.fine.pi, ref.fine.eps)
    print("coarse", info["coarse_loss_lift"], c_loss, "fine", res["loss_lift"], loss, res["egw_objective"], egw,
          "err", res["marginal_err"], info)
    assert abs(info["coarse_loss_lift"] - c_loss) <= tol * abs(c_loss)
    assert abs(res["loss_lift"] - loss) <= tol * abs(loss)
    assert abs(res["egw_objective"] - egw) <= tol * abs(egw)
    sv = np.linalg.svd(res["gamma"].cpu().numpy().astype(np.float64), compute_uv=False)
    sv_ref = np.linalg.svd(ref.fine.gamma, compute_uv=False)
    assert np.allclose(sv, sv_ref, rtol=0, atol=10 * tol * sv_ref[0])


def test_msgw_rejects_bad_options(gw):
    x, a = _gmm32(3, 200, 2)
    y, b = _gmm32(4, 150, 2)
    ctx = gw.Context()
    sched = dict(eps_start=0.1, n_outer=2, n_inner=5)
    for kw in (dict(rho=0.0), dict(rho=1.5), dict(n_lloyd=0)):
        with pytest.raises(gw.GWError):
            ctx.msgw(dev(x), dev(a), dev(y), dev(b), sched, sched, **kw)
    with pytest.raises(gw.GWError):
        ctx.msgw(dev(x), dev(a), dev(y), dev(b), dict(sched, use_init_potentials=True), sched)
    with pytest.raises(gw.GWError):
        ctx.kmeans(dev(x), dev(a), 0)
    with pytest.raises(gw.GWError):
        ctx.kmeans(dev(x), dev(a), 201)
