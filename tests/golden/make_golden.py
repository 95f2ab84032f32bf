"""Writes the stored expected values used by the GPU tests.

Every value here is computed by the FP64 oracle alone (``oracle/``) on the
seeded inputs of ``workloads``; nothing comes from the HIP library.  Run from
the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gw_oracle as O  # noqa: E402
from workloads import synth        # noqa: E402


def config1():
    """Config 1 (plain entropic GW, 512 points in the unit square, squared
    Euclidean penalty, eps = 0.01, 20 x 50 symmetric Sinkhorn)."""
    prob = synth.config1_plain()
    X, Y = O.centre(prob.x, prob.a), O.centre(prob.y, prob.b)
    res = O.cnt_gw(prob.a, prob.b, X, Y, prob.eps_start, prob.eps_end,
                   prob.n_outer, prob.n_inner)
    pi = res.pi
    cx, cy = O.sqdist(prob.x, prob.x), O.sqdist(prob.y, prob.y)
    return {
        "workload": "plain-512: x ~ U[0,1]^2, y = R x + 0.01 noise, eps 0.01, 20 x 50 symmetric",
        "loss_lift": O.lifted_loss(X, Y, prob.a, prob.b, pi),
        "loss_quartic": O.quartic_loss(cx, cy, pi),
        "kl": O.kl_divergence(pi, prob.a, prob.b),
        "egw_objective": O.egw_objective(X, Y, prob.a, prob.b, pi, res.eps),
        "marginal_error": O.marginal_error(pi, prob.a, prob.b),
        "constant_c": O.constant_c(X, Y, prob.a, prob.b),
        "gamma": res.gamma.tolist(),
        "gamma_prev": res.gamma_prev.tolist(),
        "f": res.f.tolist(),
        "g": res.g.tolist(),
    }


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_oracle.json")
    with open(out, "w") as fh:
        json.dump(config1(), fh, indent=1)
    print("wrote", out)
