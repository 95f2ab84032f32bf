"""gw_solve_noalloc against gw_solve through the C ABI: the same Algorithm 1
solve with every device buffer carved from the library's fixed scratch
array instead of allocated.  Two calls in a row (the second smaller, so it
reuses the array with the first call's contents in it) must give the
results of gw_solve bit for bit; a problem larger than the array and a
penalty that needs lifting are refused with their status codes."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2602_06658_amd import _lib as L

pytestmark = pytest.mark.gpu


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def _problem(n, m, d, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d))
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    y = x[rng.choice(n, size=m, replace=m > n)] @ q + 0.05 * rng.standard_normal((m, d))
    a = rng.dirichlet(np.ones(n) * 4)
    b = rng.dirichlet(np.ones(m) * 4)
    return dev(x), dev(a), dev(y), dev(b)


def _noalloc(ctx, x, a, y, b, prm):
    fn = ctx.lib.gw_solve_noalloc  # argument types bound from include/gw.h by the loader
    n, dx = x.shape
    m, dy = y.shape
    D, E = ctx.feature_dim(0, dx), ctx.feature_dim(1, dy)
    f = torch.empty(n, dtype=torch.float32, device="cuda")
    g = torch.empty(m, dtype=torch.float32, device="cuda")
    gamma = torch.empty((D, E), dtype=torch.float32, device="cuda")
    r = L.GwResult()
    r.f, r.g, r.gamma = f.data_ptr(), g.data_ptr(), gamma.data_ptr()
    rc = fn(ctx.h, ctypes.c_void_p(x.data_ptr()), n, dx, ctypes.c_void_p(a.data_ptr()),
            ctypes.c_void_p(y.data_ptr()), m, dy, ctypes.c_void_p(b.data_ptr()), ctypes.byref(prm), None,
            ctypes.byref(r))
    return rc, r, f, g, gamma


@pytest.mark.parametrize("prec,d", [("fp32", 3), ("fp32", 32), ("bf16", 32)])
def test_noalloc_matches_gw_solve_twice(gw, prec, d):
    from paper_2602_06658_amd.api import make_params

    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    for n, m, seed in ((3000, 2600, 1), (1100, 900, 2)):
        x, a, y, b = _problem(n, m, d, seed)
        print(f"noalloc case {prec} d={d} {n}x{m}", flush=True)
        ref = ctx.solve(x, a, y, b, 0.3, 0.05, 6, 40, precision=prec)
        prm = make_params(0.3, 0.05, 6, 40, precision=prec)
        rc, r, f, g, gamma = _noalloc(ctx, x, a, y, b, prm)
        assert rc == L.GW_OK, ctx.lib.gw_last_error(ctx.h).decode()
        for k in ("loss_lift", "egw_objective", "kl", "marginal_err", "gamma_step", "safe_iters"):
            assert getattr(r, k) == ref[k], k
        assert torch.equal(f, ref["f"]) and torch.equal(g, ref["g"]) and torch.equal(gamma, ref["gamma"])


def test_noalloc_refusals(gw):
    from paper_2602_06658_amd.api import make_params

    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    # about 1 GB of buffers for 200,000 x 200,000 at D = 64: beyond the array
    x, a, y, b = _problem(200_000, 200_000, 64, 3)
    rc, *_ = _noalloc(ctx, x, a, y, b, make_params(0.1, 0.1, 1, 1))
    assert rc == L.GW_ENOMEM
    assert "scratch" in ctx.lib.gw_last_error(ctx.h).decode()
    ctx.set_penalty(2, "power", p=1.0, lifted_dim=8, n_landmarks=64)
    x, a, y, b = _problem(500, 400, 3, 4)
    rc, *_ = _noalloc(ctx, x, a, y, b, make_params(0.1, 0.1, 1, 1))
    assert rc == L.GW_EUNSUPPORTED
