"""Inputs of the parity cases at the workloads' own schedules, shared by the
GPU tests and tests/golden/make_config_golden.py (which stores the oracle's
results for them).

Both sides of each case receive the same lifted features: the oracle's FP64
landmark kernel PCA of |x - x'| (Algorithm 4 and the Nystrom map of
Algorithm 13), rounded to single precision, so that the comparison isolates
the solver.  Centring is left to each side (the library re-centres features
it is given; the oracle's cases are re-centred in FP64)."""
from __future__ import annotations

import numpy as np

from oracle import gw_oracle as O
from workloads import config2_fp32, config3_scale, config4_requests, landmark_indices, subsample


def f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def _lifted(x, a, idx, dim):
    return f32(O.landmark_features(x, a, O.fit_landmarks(x[idx], 1.0, dim)))


def _weights(p):
    a, b = f32(p.a), f32(p.b)
    return a / a.sum(), b / b.sum()


def c3_subsample(k: int = 5000) -> dict:
    """The 200,000-point workload's seeded 5,000 + 5,000 subsample (3-D
    8-component mixture, target a noisy rigid motion), |x - x'| lifted to
    D = E = 64 with 2048 landmarks per side, eps 0.1 -> 0.005 over 30 outer
    steps of 100 symmetric Sinkhorn iterations."""
    p = subsample(config3_scale(), k, k, seed=3001)
    x, y = f32(p.x), f32(p.y)
    a, b = _weights(p)
    X = _lifted(x, a, landmark_indices(p.n, 2048, 3101), 64)
    Y = _lifted(y, b, landmark_indices(p.m, 2048, 3102), 64)
    return dict(name=f"c3sub{k}", X=X, a=a, Y=Y, b=b, eps_start=0.1, eps_end=0.005, n_outer=30, n_inner=100)


def c2_full() -> dict:
    """The 20,000-point workload (3-D 8-component mixture, target a noisy
    rigid motion), |x - x'| lifted to D = E = 32 with 2048 landmarks per
    side, eps 0.1 -> 0.005 over 30 outer steps of 100 iterations."""
    p = config2_fp32()
    x, y = f32(p.x), f32(p.y)
    a, b = _weights(p)
    X = _lifted(x, a, landmark_indices(p.n, 2048, 2101), 32)
    Y = _lifted(y, b, landmark_indices(p.m, 2048, 2102), 32)
    return dict(name="c2", X=X, a=a, Y=Y, b=b, eps_start=0.1, eps_end=0.005, n_outer=30, n_inner=100)


C4_LANDMARKS = 512


def c4_samples(count: int = 8, max_size: int = 5000):
    """The first `count` requests of the 512-request serving trace with both
    sides at most max_size points (d = 2 or 3, |x - x'| lifted to D = 32,
    eps = 0.01, 20 x 50).  Returns [(k, problem, seed)] where seed is the
    landmark seed the request carries (source seed, target seed + 1)."""
    out = []
    for k, (_, p) in enumerate(config4_requests(n_requests=512, lifted_dim=32)):
        if p.n <= max_size and p.m <= max_size:
            out.append((k, p, 7000 + 2 * k))
        if len(out) == count:
            break
    return out


def c4_features(p, seed: int):
    """Oracle features of one serving request from the library's seeded
    landmark choice (SplitMix64 Fisher-Yates, reproduced by the seeded
    inputs module)."""
    from workloads import splitmix64_landmarks

    x, y = f32(p.x), f32(p.y)
    a, b = _weights(p)
    X = _lifted(x, a, splitmix64_landmarks(p.n, C4_LANDMARKS, seed), 32)
    Y = _lifted(y, b, splitmix64_landmarks(p.m, C4_LANDMARKS, seed + 1), 32)
    return X, a, Y, b


def basin(gamma_gpu, gamma_orc, pi_argmax_gpu, pi_argmax_orc):
    """The basin check for non-convex GW: relative singular-value
    differences of the final maps and the share of rows whose argmax
    column agrees."""
    s1 = np.linalg.svd(np.asarray(gamma_gpu, np.float64), compute_uv=False)
    s2 = np.linalg.svd(np.asarray(gamma_orc, np.float64), compute_uv=False)
    sv_rel = float(np.max(np.abs(s1 - s2)) / max(s2.max(), 1e-300))
    agree = float(np.mean(np.asarray(pi_argmax_gpu) == np.asarray(pi_argmax_orc)))
    return sv_rel, agree
