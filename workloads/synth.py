"""Seeded generators for the five workloads of the hot path.

Seeds follow ``1000 * config + repetition``.  Every array is float64; the GPU
path casts to float32 itself.  The paper's own inputs are surface samples of
3-D shapes (Table 1, 4k to 177k points, uniform weights); they are not
available here, so Gaussian-mixture clouds of the same sizes stand in for
them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One GW instance: weighted source and target point sets plus settings."""

    x: np.ndarray            # (N, dx) source points
    a: np.ndarray            # (N,) source weights, positive, sum 1
    y: np.ndarray            # (M, dy) target points
    b: np.ndarray            # (M,) target weights, positive, sum 1
    eps_start: float
    eps_end: float
    n_outer: int
    n_inner: int
    penalty: str = "sqeuclid"   # "sqeuclid" | "power"
    p: float = 2.0              # exponent of |x - x'|^p for "power"
    lifted_dim: int = 0         # D = E for "power" (0: raw dimension)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def m(self) -> int:
        return self.y.shape[0]


def haar_rotation(rng: np.random.Generator, d: int) -> np.ndarray:
    """Uniform (Haar) rotation in SO(d): QR of a Gaussian matrix with the
    signs of R's diagonal moved into Q (Mezzadri 2007), then a reflection
    fix so that det = +1."""
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def gmm_points(rng: np.random.Generator, n: int, means: np.ndarray,
               sigma: float) -> np.ndarray:
    """n samples of an equal-weight isotropic Gaussian mixture."""
    k = rng.integers(0, means.shape[0], size=n)
    return means[k] + sigma * rng.standard_normal((n, means.shape[1]))


def uniform_weights(n: int) -> np.ndarray:
    return np.full(n, 1.0 / n)


def rotated_copy(rng: np.random.Generator, x: np.ndarray, noise: float,
                 translate: bool) -> np.ndarray:
    """y = R x + t + noise * xi with R Haar, t ~ U[-1,1]^d (if translate)."""
    d = x.shape[1]
    rot = haar_rotation(rng, d)
    t = rng.uniform(-1.0, 1.0, size=d) if translate else np.zeros(d)
    return x @ rot.T + t[None, :] + noise * rng.standard_normal(x.shape)


def config1_plain(rep: int = 0, n: int = 512) -> Problem:
    """Plain entropic GW, squared-Euclidean penalty: x ~ U[0,1]^2, y = source
    rotated by a uniform angle plus N(0, 0.01^2) noise, uniform weights,
    eps = 0.01, 20 outer x 50 symmetric Sinkhorn iterations."""
    rng = np.random.default_rng(1000 * 1 + rep)
    x = rng.uniform(0.0, 1.0, size=(n, 2))
    theta = rng.uniform(0.0, 2.0 * np.pi)
    rot = np.array([[np.cos(theta), -np.sin(theta)],
                    [np.sin(theta), np.cos(theta)]])
    y = x @ rot.T + 0.01 * rng.standard_normal((n, 2))
    return Problem(x, uniform_weights(n), y, uniform_weights(n),
                   0.01, 0.01, 20, 50, "sqeuclid", 2.0, 0, "plain-512",
                   {"theta": theta})


def _gmm_pair(seed: int, n: int, d: int, k: int, sigma: float,
              noise: float) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(k, d))
    x = gmm_points(rng, n, means, sigma)
    y = rotated_copy(rng, x, noise, translate=True)
    return x, y


def config2_fp32(rep: int = 0, n: int = 20_000, lifted_dim: int = 32) -> Problem:
    """3-D 8-component mixture (means U[-1,1]^3, sigma 0.1); target = Haar
    rotation + translation + N(0, 0.005^2) noise; |x - x'| penalty lifted to
    D = 32; eps annealed 0.1 -> 0.005 over 30 outer steps, 100 inner."""
    x, y = _gmm_pair(1000 * 2 + rep, n, 3, 8, 0.1, 0.005)
    return Problem(x, uniform_weights(n), y, uniform_weights(n),
                   0.1, 0.005, 30, 100, "power", 1.0, lifted_dim,
                   f"gmm3d-{n}")


def config3_scale(rep: int = 0, n: int = 200_000, lifted_dim: int = 64) -> Problem:
    """Same generator as config 2 at N = M = 200,000 with D = 64."""
    x, y = _gmm_pair(1000 * 3 + rep, n, 3, 8, 0.1, 0.005)
    return Problem(x, uniform_weights(n), y, uniform_weights(n),
                   0.1, 0.005, 30, 100, "power", 1.0, lifted_dim,
                   f"gmm3d-{n}")


def config4_requests(n_requests: int = 512, lo: int = 1_000, hi: int = 50_000,
                     lifted_dim: int = 32, seed_base: int = 4000,
                     rate: float = 1.0) -> list[tuple[float, Problem]]:
    """Serving trace: sizes log-uniform in [lo, hi] drawn independently for
    source and target, dimension 2 or 3 with probability 1/2 each, source and
    target are independent samples of one 8-component mixture with the target
    under a Haar rigid motion; eps = 0.01, 20 outer x 50 inner.  Arrival
    times are a Poisson process of the given rate (requests per second)."""
    trace_rng = np.random.default_rng(seed_base - 1)
    gaps = trace_rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_requests):
        rng = np.random.default_rng(seed_base + k)
        n = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        m = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        d = 2 if rng.uniform() < 0.5 else 3
        means = rng.uniform(-1.0, 1.0, size=(8, d))
        x = gmm_points(rng, n, means, 0.1)
        y0 = gmm_points(rng, m, means, 0.1)
        y = rotated_copy(rng, y0, 0.0, translate=True)
        out.append((float(arrivals[k]),
                    Problem(x, uniform_weights(n), y, uniform_weights(m),
                            0.01, 0.01, 20, 50, "power", 1.0, lifted_dim,
                            f"req{k}-{n}x{m}-d{d}")))
    return out


def config5_grad(rep: int = 0, n: int = 50_000, m: int = 30_000,
                 lifted_dim: int = 64) -> Problem:
    """d = 16, 16-component mixture (means U[-1,1]^16, sigma 0.1); source and
    target are independent draws of the mixture (target under a rigid
    motion); weights Dirichlet(1); |x - x'| lifted to D = 64; eps = 0.01,
    20 outer x 50 inner."""
    rng = np.random.default_rng(1000 * 5 + rep)
    means = rng.uniform(-1.0, 1.0, size=(16, 16))
    x = gmm_points(rng, n, means, 0.1)
    y0 = gmm_points(rng, m, means, 0.1)
    y = rotated_copy(rng, y0, 0.0, translate=True)
    a = rng.dirichlet(np.ones(n))
    b = rng.dirichlet(np.ones(m))
    return Problem(x, a, y, b, 0.01, 0.01, 20, 50, "power", 1.0, lifted_dim,
                   f"grad-{n}x{m}-d16")


def grad_points(seed: int, n: int, m: int, d: int, noise: float = 0.05, scale: float = 1.0):
    """Small gradient-parity inputs: x ~ N(0, scale^2 I_d); y = an orthogonal
    image of a random subset of x plus N(0, noise^2) noise; weights
    Dirichlet(3), rounded to float32 and renormalised in float64.  Returns
    float32-representable float64 arrays (x, a, y, b)."""
    rng = np.random.default_rng(seed)
    x = scale * rng.standard_normal((n, d))
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    y = x[rng.choice(n, m, replace=False)] @ q + noise * rng.standard_normal((m, d))
    f32 = lambda v: np.asarray(v, dtype=np.float32).astype(np.float64)  # noqa: E731
    a = f32(rng.dirichlet(np.ones(n) * 3))
    b = f32(rng.dirichlet(np.ones(m) * 3))
    return f32(x), a / a.sum(), f32(y), b / b.sum()


def c5_subsample(n_src: int, n_tgt: int, seed: int):
    """A seeded subsample of the differentiation workload (50,000 x 30,000,
    d = 16, Dirichlet weights), rounded to float32 with the weights
    renormalised in float64.  Returns (x, a, y, b)."""
    sub = subsample(config5_grad(), n_src, n_tgt, seed)
    f32 = lambda v: np.asarray(v, dtype=np.float32).astype(np.float64)  # noqa: E731
    a, b = f32(sub.a), f32(sub.b)
    return f32(sub.x), a / a.sum(), f32(sub.y), b / b.sum()


def scale_features(seed: int, n: int, d: int, decay: float = 1.5) -> np.ndarray:
    """Feature clouds shaped like landmark kernel-PCA features: independent
    Gaussian coordinates with variances proportional to k^-decay
    (k = 1..d), total variance 1.  Float32-representable float64."""
    rng = np.random.default_rng(seed)
    var = np.arange(1, d + 1, dtype=np.float64) ** -decay
    var /= var.sum()
    x = rng.standard_normal((n, d)) * np.sqrt(var)[None, :]
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def seeded_gamma(seed: int, d: int, e: int, scale: float = 0.5) -> np.ndarray:
    """A D x E starting map: scale times the first rows/columns of a Haar
    orthogonal matrix.  Float32-representable float64."""
    q = haar_rotation(np.random.default_rng(seed), max(d, e))[:d, :e]
    return np.asarray(scale * q, dtype=np.float32).astype(np.float64)


def landmark_indices(n: int, n_landmarks: int, seed: int) -> np.ndarray:
    """Landmark subset for kernel PCA: the first n_l entries of a seeded
    permutation, sorted.  A random draw of the method, so both the oracle and
    the GPU path receive it as an input."""
    perm = np.random.default_rng(seed).permutation(n)
    return np.sort(perm[: min(n_landmarks, n)])


_MASK64 = (1 << 64) - 1


def splitmix64_stream(seed: int):
    """SplitMix64 (Steele, Lea, Flood 2014): state += 0x9E3779B97F4A7C15,
    output = the state through two xor-shift-multiply rounds and a final
    xor-shift."""
    state = seed & _MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        yield z ^ (z >> 31)


def splitmix64_landmarks(n: int, n_landmarks: int, seed: int) -> np.ndarray:
    """The seeded landmark choice for requests that carry a seed instead of
    indices: a Fisher-Yates shuffle of 0..n-1 (i from n-1 down to 1 swaps
    with j = next() mod (i + 1)), first n_landmarks entries, sorted.  A random
    draw of the method, so both the library and the oracle's inputs use this
    one published generator."""
    perm = list(range(n))
    gen = splitmix64_stream(seed)
    for i in range(n - 1, 0, -1):
        j = next(gen) % (i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return np.sort(np.array(perm[: min(n_landmarks, n)], dtype=np.int64))


def subsample(prob: Problem, k_src: int, k_tgt: int, seed: int) -> Problem:
    """Seeded subsample of both clouds; weights renormalised to sum 1."""
    rng = np.random.default_rng(seed)
    i = np.sort(rng.choice(prob.n, size=min(k_src, prob.n), replace=False))
    j = np.sort(rng.choice(prob.m, size=min(k_tgt, prob.m), replace=False))
    a = prob.a[i] / prob.a[i].sum()
    b = prob.b[j] / prob.b[j].sum()
    return Problem(prob.x[i], a, prob.y[j], b, prob.eps_start, prob.eps_end,
                   prob.n_outer, prob.n_inner, prob.penalty, prob.p,
                   prob.lifted_dim, prob.name + f"-sub{len(i)}x{len(j)}",
                   {"rows": i, "cols": j})
