"""Write tests/golden/grad_*.json: the FP64 oracle's converged CNT-GW
solution and its envelope gradients (Appendix B.6) for the seeded inputs of
workloads.grad_points.  Calls only oracle/ and workloads/.

Each case: a fixed-schedule Algorithm 1 run, then the converged solve
(Sinkhorn to 1e-13 marginal error per outer step, outer steps until
|Gamma_{t+1} - Gamma_t| is below the case's tolerance) warm-started from it.  Stored: Gamma*
(in the oracle's feature basis), the loss, the final marginal error and the
converged potentials f*, g* (Algorithm 1's convention), and the
four gradients (positions through centring and, for the |x - x'| penalty,
the frozen Nystrom map; weights as the converged potential of the full
linearised cost, centred).

    python tests/golden/make_grad_golden.py [case ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import gw_oracle as O  # noqa: E402
from workloads import c5_subsample, grad_points, landmark_indices  # noqa: E402

CASES = {
    # name: (seed, n, m, d, penalty, lifted_dim, n_landmarks, eps, outer tolerance)
    "sqeuclid": (60, 200, 170, 3, "sqeuclid", 0, 0, 0.3, 1e-11),
    "power16": (61, 230, 190, 3, "power", 16, 96, 0.3, 1e-11),
    # 40-dimensional features scaled to norms of order 1 (see SCALE)
    "features40": (62, 200, 170, 40, "features", 0, 0, 0.3, 1e-10),
    # a subsample of the differentiation workload (d = 16, Dirichlet weights,
    # |x - x'| lifted to D = 64); eps 0.05 so that the FP64 reference converges
    "c5sub": (65, 300, 250, 16, "power", 64, 128, 0.05, 1e-10),
}
# cases whose inputs come from workloads.c5_subsample instead of grad_points
C5 = {"c5sub"}
# input scale per case: N(0, I_d) points have |x|^2 ~ d, and a cost range of
# hundreds against eps / 8 makes every converged Sinkhorn solve crawl
SCALE = {"features40": 40 ** -0.5}


def features(case):
    seed, n, m, d, pen, D, nl, eps, _ = CASES[case]
    if case in C5:
        x, a, y, b = c5_subsample(n, m, seed)
    else:
        x, a, y, b = grad_points(seed, n, m, d, noise=0.02 if pen == "power" else 0.05, scale=SCALE.get(case, 1.0))
    if pen == "power":
        ix, iy = landmark_indices(n, nl, seed + 1), landmark_indices(m, nl, seed + 2)
        lmx, lmy = O.fit_landmarks(x[ix], 1.0, D), O.fit_landmarks(y[iy], 1.0, D)
        return x, a, y, b, O.landmark_features(x, a, lmx), O.landmark_features(y, b, lmy), (ix, iy, lmx, lmy)
    return x, a, y, b, O.centre(x, a), O.centre(y, b), None


def run(case):
    seed, n, m, d, pen, D, nl, eps, tol = CASES[case]
    x, a, y, b, X, Y, lm = features(case)
    t0 = time.time()
    r = O.cnt_gw(a, b, X, Y, eps, eps, 40, 200)
    gam, pi, f, g = O.cnt_gw_converged(a, b, X, Y, eps, gamma0=r.gamma, tol=tol, sink_tol=1e-13)
    gfx = O.chain_centre(O.grad_features(X, Y, a, b, pi, gam), a)
    gfy = O.chain_centre(O.grad_features_target(X, Y, a, b, pi, gam), b)
    if lm is not None:
        gfx = np.einsum("nd,ndk->nk", gfx, O.kernel_proj_jacobian(x, lm[2]))
        gfy = np.einsum("nd,ndk->nk", gfy, O.kernel_proj_jacobian(y, lm[3]))
    ga = O.grad_weights(O.sqdist(X, X), O.sqdist(Y, Y), a, b, pi, eps)
    gb = O.grad_weights(O.sqdist(Y, Y), O.sqdist(X, X), b, a, pi.T, eps)
    out = {
        "case": case, "seed": seed, "n": n, "m": m, "d": d, "penalty": pen, "lifted_dim": D,
        "n_landmarks": nl, "eps": eps, "outer_tol": tol, "scale": SCALE.get(case, 1.0),
        "inputs": "c5_subsample" if case in C5 else "grad_points",
        "landmarks_x": None if lm is None else lm[0].tolist(),
        "landmarks_y": None if lm is None else lm[1].tolist(),
        "gamma": gam.tolist(), "f": f.tolist(), "g": g.tolist(), "loss_lift": O.lifted_loss(X, Y, a, b, pi),
        "egw_objective": O.egw_objective(X, Y, a, b, pi, eps),
        "marginal_error": O.marginal_error(pi, a, b),
        "grad_x": gfx.tolist(), "grad_y": gfy.tolist(), "grad_a": ga.tolist(), "grad_b": gb.tolist(),
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, f"grad_{case}.json"), "w") as fh:
        json.dump(out, fh)
    print(case, "done in %.0f s, Err %.2e" % (out["oracle_seconds"], out["marginal_error"]), flush=True)


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        run(c)
