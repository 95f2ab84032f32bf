"""Write the oracle's results for the parity cases at the workloads' own
schedules (inputs from tests/config_cases.py).  Calls only oracle/ and
workloads/ (through config_cases).

    python tests/golden/make_config_golden.py c3sub   # c3sub5000_oracle.json (~10 min)
    python tests/golden/make_config_golden.py c3sub_inputs   # c3sub5000_inputs.npz
    python tests/golden/make_config_golden.py c4      # c4_samples_oracle.json
    python tests/golden/make_config_golden.py c2      # c2_oracle.json + .npz (~1.5 h)

Every case runs Algorithm 1 in FP64 with the oracle's C Sinkhorn loop
(equal to its NumPy loop to float64 rounding, pinned in
tests/test_oracle_sinkhorn_c.py).  Stored per case: the Lemma C.1 loss, EGW
objective, KL, marginal error, Gamma_T and its singular values, the argmax
column of every row of the final coupling, and fingerprints of the features
(norms) so a test can tell that it rebuilt the same inputs.  The 5,000-point
case also stores the final potentials, Gamma_{T-1}, and one further
symmetric Sinkhorn iteration from that state at the last temperature, with
the single-precision error bounds of that one step (see
tests/test_gpu_config_schedules.py).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import config_cases as CC  # noqa: E402
from oracle import gw_oracle as O  # noqa: E402


def summary(case, X, Y, a, b, ref, t0):
    pi = ref.pi
    loss = O.lifted_loss(X, Y, a, b, pi)
    kl = O.kl_divergence(pi, a, b)
    return {"name": case["name"], "n": int(X.shape[0]), "m": int(Y.shape[0]), "D": int(X.shape[1]),
            "E": int(Y.shape[1]), "eps_start": case["eps_start"], "eps_end": case["eps_end"],
            "n_outer": case["n_outer"], "n_inner": case["n_inner"], "eps_final": ref.eps,
            "loss_lift": loss, "egw_objective": loss + ref.eps * kl, "kl": kl,
            "marginal_error": O.marginal_error(pi, a, b), "gamma": ref.gamma.tolist(),
            "gamma_sv": np.linalg.svd(ref.gamma, compute_uv=False).tolist(),
            "argmax_rows": np.argmax(pi, axis=1).tolist(),
            "feature_norms": [float(np.linalg.norm(case["X"])), float(np.linalg.norm(case["Y"]))],
            "oracle_seconds": time.time() - t0}


def one_step_bounds(X, Y, a, b, gamma, f, g, eps):
    """One symmetric Sinkhorn iteration from (f, g) with the map gamma at
    eps, and the bounds a single-precision evaluation of it is held to: each
    exponent (log2 units, kappa = log2(e) / eps') is assembled from terms of
    magnitude at most S, a few roundings give |ds| <= 16 ulp(S), and the
    potential moves by at most (eps'/2) ln 2 * 16 * 2^-24 * S; BF16 feature
    products add 2^-8 sum_k |X_ik| max_j |Z_jk| (1-Lipschitz log-sum-exp)."""
    epsp = eps / 8.0
    xbar = O.lift(X)
    z = Y @ gamma.T
    zbar = np.concatenate([z, 0.5 * np.sum(Y * Y, 1, keepdims=True)], 1)
    c = O.sqdist(xbar, zbar)
    f1, g1 = O.sinkhorn(a, b, c, epsp, 1, f, g, True, backend="c")
    kappa = np.log2(np.e) / epsp
    n2, m2 = np.sum(X * X, 1), np.sum(Y * Y, 1)
    alpha, beta = n2 + 0.25 * n2 ** 2, np.sum(z * z, 1) + 0.25 * m2 ** 2
    fh, gh = np.abs(f - alpha), np.abs(g - beta)
    zabs, xabs = np.abs(z).max(0), np.abs(X).max(0)
    s_row = kappa * (fh + gh.max() + alpha + beta.max() + 2 * np.abs(X) @ zabs + 0.5 * n2 * m2.max() + c.max(1))
    s_col = kappa * (fh.max() + gh + alpha.max() + beta + 2 * np.abs(z) @ xabs + 0.5 * n2.max() * m2 + c.max(0))
    fp32 = lambda s: 0.5 * epsp * np.log(2) * 16 * 2.0 ** -24 * s  # noqa: E731
    return {"f1": f1.tolist(), "g1": g1.tolist(), "tol_fp32_rows": fp32(s_row).tolist(),
            "tol_fp32_cols": fp32(s_col).tolist(), "tol_bf16_rows": (2.0 ** -8 * np.abs(X) @ zabs).tolist(),
            "tol_bf16_cols": (2.0 ** -8 * np.abs(z) @ xabs).tolist()}


def solve_case(case):
    a, b = case["a"], case["b"]
    X, Y = O.centre(case["X"], a), O.centre(case["Y"], b)
    ref = O.cnt_gw(a, b, X, Y, case["eps_start"], case["eps_end"], case["n_outer"], case["n_inner"], backend="c")
    return X, Y, ref


def c3sub():
    t0 = time.time()
    case = CC.c3_subsample()
    X, Y, ref = solve_case(case)
    out = summary(case, X, Y, case["a"], case["b"], ref, t0)
    out.update({"f": ref.f.tolist(), "g": ref.g.tolist(), "gamma_prev": ref.gamma_prev.tolist()})
    out["one_step"] = one_step_bounds(X, Y, case["a"], case["b"], ref.gamma_prev, ref.f, ref.g, ref.eps)
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, f"{case['name']}_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print(f"{case['name']}: loss {out['loss_lift']:.10g} err {out['marginal_error']:.3e} "
          f"({out['oracle_seconds']:.0f} s)", flush=True)


def c3sub_inputs():
    """The 5,000-point case's single-precision features and weights (what
    the GPU receives), for the bench's parity leg and its CPU baseline,
    which do not rebuild them with the oracle's kernel PCA."""
    case = CC.c3_subsample()
    np.savez_compressed(os.path.join(HERE, f"{case['name']}_inputs.npz"), X=case["X"].astype(np.float32),
                        a=case["a"].astype(np.float32), Y=case["Y"].astype(np.float32),
                        b=case["b"].astype(np.float32))
    print(f"{case['name']} inputs written", flush=True)


def c2():
    t0 = time.time()
    case = CC.c2_full()
    X, Y, ref = solve_case(case)
    out = summary(case, X, Y, case["a"], case["b"], ref, t0)
    amax = np.array(out.pop("argmax_rows"), dtype=np.int32)
    np.savez_compressed(os.path.join(HERE, "c2_oracle.npz"), f=ref.f.astype(np.float32),
                        g=ref.g.astype(np.float32), argmax_rows=amax)
    with open(os.path.join(HERE, "c2_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print(f"c2: loss {out['loss_lift']:.10g} err {out['marginal_error']:.3e} ({out['oracle_seconds']:.0f} s)",
          flush=True)


def c4():
    res = []
    for k, p, seed in CC.c4_samples():
        t0 = time.time()
        X, a, Y, b = CC.c4_features(p, seed)
        case = dict(name=f"req{k}", X=X, a=a, Y=Y, b=b, eps_start=p.eps_start, eps_end=p.eps_end,
                    n_outer=p.n_outer, n_inner=p.n_inner)
        Xc, Yc, ref = solve_case(case)
        s = summary(case, Xc, Yc, a, b, ref, t0)
        s.update({"request": k, "seed": seed, "dx": int(p.x.shape[1])})
        res.append(s)
        print(f"request {k} ({p.n}x{p.m}, d={p.x.shape[1]}): loss {s['loss_lift']:.8g} "
              f"err {s['marginal_error']:.2e} ({s['oracle_seconds']:.0f} s)", flush=True)
    with open(os.path.join(HERE, "c4_samples_oracle.json"), "w") as fh:
        json.dump({"landmarks": CC.C4_LANDMARKS, "requests": res}, fh)


if __name__ == "__main__":
    for what in sys.argv[1:] or ["c3sub", "c4"]:
        {"c3sub": c3sub, "c3sub_inputs": c3sub_inputs, "c2": c2, "c4": c4}[what]()
