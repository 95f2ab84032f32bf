"""Algorithm 6's adaptive Sinkhorn counts on the GPU (gw_params.adaptive_inner)
against the oracle's CNT-GW with the paper's rule (double on any increase of
the EGW objective beyond float64 rounding): the same doublings, the same
final count, the EGW objective within the FP32 loss tolerance 1e-5.

The GPU doubles only on increases above 1e-6 max(|EGW|, C), its
single-precision tolerance.  The cases are chosen so that the two rules take
the same decisions: every increase of the objective between outer steps in
the oracle's run is above 2.5e-6 of the scale, and no count reaches the
GPU's cap of 64 n_inner (the oracle records each comparison, and the test
checks this before comparing).  A case where the rules differ is pinned on
the CPU (test_oracle_adaptive.py).  The server rejects the mode."""
import numpy as np
import pytest
import torch

from oracle import gw_oracle as O

pytestmark = pytest.mark.gpu


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def _case(seed, n, m, d):
    rng = np.random.default_rng(seed)
    s = np.sqrt(2.0 / d)
    x = (rng.standard_normal((n, d)) * np.linspace(1.0, 0.5, d) * s).astype(np.float32).astype(np.float64)
    y = (rng.standard_normal((m, d)) * np.linspace(0.9, 0.6, d) * s).astype(np.float32).astype(np.float64)
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    return x, a, y, b


@pytest.mark.parametrize("seed,n,m,d,eps,T,nin", [(5, 300, 260, 2, 0.3, 40, 1), (6, 300, 260, 2, 0.1, 30, 2),
                                                  (11, 400, 350, 16, 0.5, 20, 2)])
def test_adaptive_counts_match_oracle(gw, seed, n, m, d, eps, T, nin):
    x, a, y, b = _case(seed, n, m, d)
    ctx = gw.Context()
    if d >= 16:
        ctx.set_penalty(2, "features")
    print(f"adaptive seed={seed} n={n} m={m} d={d} eps={eps} T={T} n_inner={nin}", flush=True)
    res = ctx.solve(dev(x), dev(a), dev(y), dev(b), eps, eps, T, nin, precision="fp32", adaptive_inner=True)
    X, Y = O.centre(x, a), O.centre(y, b)
    ref = O.cnt_gw(a, b, X, Y, eps, eps, T, nin, adaptive=True)
    ratios = [(e1 - e0) / sc for (_, e1, e0, sc, _) in ref.adaptive_log]
    assert not [q for q in ratios if O.ADAPTIVE_TIE < q <= 2.5e-6], ratios
    assert ref.n_inner_final <= 64 * nin
    egw = O.egw_objective(X, Y, a, b, ref.pi, ref.eps)
    print(res["inner_doublings"], ref.doublings, res["n_inner_final"], ref.n_inner_final, res["egw_objective"], egw)
    assert res["inner_doublings"] == ref.doublings and res["n_inner_final"] == ref.n_inner_final
    assert abs(res["egw_objective"] - egw) <= 1e-5 * abs(egw)


def test_fixed_counts_report_no_doublings(gw):
    x, a, y, b = _case(8, 200, 180, 2)
    res = gw.Context().solve(dev(x), dev(a), dev(y), dev(b), 0.3, 0.3, 5, 7)
    assert res["inner_doublings"] == 0 and res["n_inner_final"] == 7


def test_server_rejects_adaptive(gw):
    x, a, y, b = _case(9, 100, 90, 2)
    srv = gw.Server(gw.Context(), max_slots=2)
    try:
        with pytest.raises(gw.GWError):
            srv.wait(srv.submit(dev(x), dev(a), dev(y), dev(b), 0.3, 0.3, 3, 5, adaptive_inner=True))
    finally:
        srv.close()
