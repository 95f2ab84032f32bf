"""Write tests/golden/scale200k_eps*.json: one symmetric Sinkhorn iteration
(Algorithm 3) of the FP64 oracle at 200,000 x 200,000, D = E = 64, from the
seeded state (workloads.scale_features, workloads.seeded_gamma, f = g = 0),
evaluated for 4096 sampled rows and 4096 sampled columns over all their
counterparts, plus the error bounds the GPU result is held to (see
tests/test_gpu_scale.py).  Calls only oracle/ and workloads/.

    python tests/golden/make_scale_golden.py [eps ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import gw_oracle as O  # noqa: E402
from workloads import scale_features, seeded_gamma  # noqa: E402

N = M = 200_000
D = 64
SAMPLES = 4096
BLOCK = 256
SEEDS = dict(x=3301, y=3302, gamma=3303, sample=3304)


def inputs():
    x = scale_features(SEEDS["x"], N, D)
    y = scale_features(SEEDS["y"], M, D)
    gam = seeded_gamma(SEEDS["gamma"], D, D)
    return x, np.full(N, 1.0 / N), y, np.full(M, 1.0 / M), gam


def run(eps):
    t0 = time.time()
    x, a, y, b, gam = inputs()
    X, Y = O.centre(x, a), O.centre(y, b)
    xbar = O.lift(X)
    z = Y @ gam.T
    zbar = np.concatenate([z, 0.5 * np.sum(Y * Y, 1, keepdims=True)], 1)
    rng = np.random.default_rng(SEEDS["sample"])
    rows = np.sort(rng.choice(N, SAMPLES, replace=False))
    cols = np.sort(rng.choice(M, SAMPLES, replace=False))
    epsp = eps / 8.0
    f1, g1 = np.empty(SAMPLES), np.empty(SAMPLES)
    cmax_r, cmax_c = np.empty(SAMPLES), np.empty(SAMPLES)
    zero_m, zero_n = np.zeros(M), np.zeros(N)
    for s0 in range(0, SAMPLES, BLOCK):
        c = O.sqdist(xbar[rows[s0:s0 + BLOCK]], zbar)
        f1[s0:s0 + BLOCK] = 0.5 * O.softmin_rows(b, zero_m, c, epsp)
        cmax_r[s0:s0 + BLOCK] = c.max(1)
        c = O.sqdist(xbar, zbar[cols[s0:s0 + BLOCK]])
        g1[s0:s0 + BLOCK] = 0.5 * O.softmin_cols(a, zero_n, c, epsp)
        cmax_c[s0:s0 + BLOCK] = c.max(0)
        print(f"eps {eps}: {s0 + BLOCK}/{SAMPLES} ({time.time() - t0:.0f} s)", flush=True)
    # bounds (log2 exponent units, kappa = log2(e) / eps')
    kappa = np.log2(np.e) / epsp
    n2, m2 = np.sum(X * X, 1), np.sum(Y * Y, 1)
    alpha, beta = n2 + 0.25 * n2 ** 2, np.sum(z * z, 1) + 0.25 * m2 ** 2
    zabs, xabs = np.abs(z).max(0), np.abs(X).max(0)
    s_row = kappa * (alpha[rows] + beta.max() + 2 * np.abs(X[rows]) @ zabs + 0.5 * n2[rows] * m2.max() + cmax_r)
    s_col = kappa * (alpha.max() + beta[cols] + 2 * np.abs(z[cols]) @ xabs + 0.5 * n2.max() * m2[cols] + cmax_c)
    fp32 = lambda s: 0.5 * epsp * np.log(2) * 16 * 2.0 ** -24 * s  # noqa: E731
    out = {"eps": eps, "n": N, "m": M, "d": D, "seeds": SEEDS, "rows": rows.tolist(), "cols": cols.tolist(),
           "f1": f1.tolist(), "g1": g1.tolist(),
           "tol_fp32_rows": fp32(s_row).tolist(), "tol_fp32_cols": fp32(s_col).tolist(),
           "tol_bf16_rows": (2.0 ** -8 * np.abs(X[rows]) @ zabs).tolist(),
           "tol_bf16_cols": (2.0 ** -8 * np.abs(z[cols]) @ xabs).tolist(),
           "oracle_seconds": time.time() - t0}
    with open(os.path.join(HERE, f"scale200k_eps{eps:g}.json"), "w") as fh:
        json.dump(out, fh)
    print(f"eps {eps} done in {out['oracle_seconds']:.0f} s", flush=True)


if __name__ == "__main__":
    for e in (sys.argv[1:] or ["4.0", "1.0", "0.1"]):
        run(float(e))
