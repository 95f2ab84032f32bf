"""Multi-seed landscape workload (random Gamma_0 for one pair, the paper's
exploration of GW local minima from hundreds of initialisations) through
the serving loop: each served solve against the FP64 oracle started from
the same Gamma_0 (a random draw of the method, passed to both sides), and
bitwise against gw_solve alone."""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as O
from workloads import gmm_points, rotated_copy, seeded_gamma

pytestmark = pytest.mark.gpu


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def f32(v):
    return np.asarray(v, dtype=np.float32).astype(np.float64)


def test_random_initialisations_through_the_server(gw):
    rng = np.random.default_rng(8100)
    means = rng.uniform(-1.0, 1.0, size=(6, 3))
    x = f32(gmm_points(rng, 400, means, 0.15))
    y = f32(rotated_copy(rng, gmm_points(rng, 360, means, 0.15), 0.0, translate=True))
    a, b = np.full(400, 1.0 / 400), np.full(360, 1.0 / 360)
    eps, n_outer, n_inner = 0.05, 10, 50
    gammas = [f32(seeded_gamma(7000 + k, 3, 3, scale=1.0)) for k in range(8)]
    srv = gw.Server(gw.Context(), max_slots=4)
    tickets = [srv.submit(dev(x), dev(a), dev(y), dev(b), eps, eps, n_outer, n_inner, gamma0=dev(g0))
               for g0 in gammas]
    outs = [srv.wait(t) for t in tickets]
    srv.close()
    X, Y = O.centre(x, a), O.centre(y, b)
    losses = []
    for k, (g0, out) in enumerate(zip(gammas, outs)):
        ref = O.cnt_gw(a, b, X, Y, eps, eps, n_outer, n_inner, gamma0=g0)
        ref_loss = O.lifted_loss(X, Y, a, b, ref.pi)
        rel = abs(out["loss_lift"] - ref_loss) / abs(ref_loss)
        losses.append(ref_loss)
        print(f"seed {k}: loss {out['loss_lift']:.8g} oracle {ref_loss:.8g} rel {rel:.2e}")
        assert rel < 1e-5
    print("distinct minima (loss to 1e-4):", len(np.unique(np.round(np.array(losses), 4))))
    ctx = gw.Context()
    for k in (0, 5):
        alone = ctx.solve(dev(x), dev(a), dev(y), dev(b), eps, eps, n_outer, n_inner, gamma0=dev(gammas[k]))
        for key in ("f", "g", "gamma"):
            assert torch.equal(alone[key], outs[k][key]), (k, key)
