"""Error paths and the stepwise solve of the C ABI (include/gw.h), on the GPU.

Validation follows the problem statement of Section 5 ("Notations"): two
weighted point sets with positive weights summing to one, a temperature
eps > 0 and iteration counts >= 1.  Every rejected call must return its
status without launching work that could fault; the numeric failure is
forced from the host (a forced single-exponential mode on a cold start whose
sums underflow), so every kernel still exits normally.

The stepwise entry points keep Algorithm 1's state (f, g, Gamma_t, t) in
the context: begin + advance(k1) + advance(k2) + end must equal gw_solve bit
for bit.  A warm start through the public outputs (Gamma_t, f, g in single
precision) resumes the same iteration up to that rounding."""
import numpy as np
import pytest
import torch

from paper_2602_06658_amd import _lib as L

pytestmark = pytest.mark.gpu


def dev(v):
    return torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")


def _problem(n=300, m=260, d=3, seed=5, scale=1.0):
    rng = np.random.default_rng(seed)
    x = scale * rng.standard_normal((n, d))
    y = scale * rng.standard_normal((m, d))
    a = rng.dirichlet(np.ones(n) * 4)
    b = rng.dirichlet(np.ones(m) * 4)
    return x, a, y, b


def _code(excinfo):
    return excinfo.value.code


@pytest.mark.parametrize("entry", ["solve", "loss_and_grad"])
def test_invalid_inputs_are_rejected(gw, entry):
    x, a, y, b = _problem()
    ctx = gw.Context()
    ctx.set_penalty(2, "sqeuclid")

    def call(x_, a_, y_, b_, eps=0.1, n_outer=2, n_inner=5, **kw):
        if entry == "solve":
            return ctx.solve(dev(x_), dev(a_), dev(y_), dev(b_), eps, eps, n_outer, n_inner, **kw)
        return ctx.loss_and_grad(dev(x_), dev(a_), dev(y_), dev(b_), eps, eps, n_outer, n_inner, **kw)

    call(x, a, y, b)  # the valid problem runs
    bad_x = x.copy()
    bad_x[7, 1] = np.nan
    inf_y = y.copy()
    inf_y[3, 0] = np.inf
    neg_a = a.copy()
    neg_a[0], neg_a[1] = -neg_a[0], neg_a[1] + 2 * neg_a[0]
    cases = [
        ("NaN in x", dict(x_=bad_x)),
        ("Inf in y", dict(y_=inf_y)),
        ("negative weight", dict(a_=neg_a)),
        ("weights sum to 1 + 3e-6", dict(a_=a * (1 + 3e-6))),
        ("NaN weight", dict(b_=np.where(np.arange(len(b)) == 4, np.nan, b))),
        ("eps = 0", dict(eps=0.0)),
        ("eps < 0", dict(eps=-0.1)),
        ("n_outer = 0", dict(n_outer=0)),
        ("n_inner = 0", dict(n_inner=0)),
    ]
    for name, kw in cases:
        args = dict(x_=x, a_=a, y_=y, b_=b)
        args.update({k: v for k, v in kw.items() if k.endswith("_")})
        extra = {k: v for k, v in kw.items() if not k.endswith("_")}
        with pytest.raises(L.GWError) as ei:
            call(**args, **extra)
        assert _code(ei) == L.GW_EINVAL, name
    # within the stated tolerance the FP64 sum is accepted
    call(x, a * (1 + 5e-7), y, b)


def test_dimension_and_size_limits(gw):
    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    rng = np.random.default_rng(1)
    w = np.full(40, 1 / 40)
    with pytest.raises(L.GWError) as ei:  # D > 256
        ctx.solve(dev(rng.standard_normal((40, 257))), dev(w), dev(rng.standard_normal((40, 4))), dev(w), 0.1)
    assert _code(ei) == L.GW_EINVAL
    with pytest.raises(L.GWError) as ei:  # n < 1: no points
        ctx.solve(dev(np.zeros((0, 3))), dev(np.zeros(0)), dev(rng.standard_normal((40, 3))), dev(w), 0.1)
    assert _code(ei) == L.GW_EINVAL
    with pytest.raises(L.GWError) as ei:  # unknown precision
        ctx.solve(dev(rng.standard_normal((40, 3))), dev(w), dev(rng.standard_normal((40, 3))), dev(w), 0.1,
                  precision=7)
    assert _code(ei) == L.GW_EINVAL


def test_workspace_limit_gives_enomem(gw):
    x, a, y, b = _problem(n=4000, m=3000, d=32)
    ctx = gw.Context(workspace_limit=1 << 20)
    ctx.set_penalty(2, "features")
    with pytest.raises(L.GWError) as ei:
        ctx.solve(dev(x), dev(a), dev(y), dev(b), 0.1, 0.1, 1, 2)
    assert _code(ei) == L.GW_ENOMEM
    # the same context solves once the limit allows it
    ctx2 = gw.Context(workspace_limit=1 << 30)
    ctx2.set_penalty(2, "features")
    r = ctx2.solve(dev(x), dev(a), dev(y), dev(b), 0.1, 0.1, 1, 2)
    assert np.isfinite(r["loss_lift"])


@pytest.mark.parametrize("d", [2, 32])
def test_forced_single_exponential_cold_start_is_a_numeric_error(gw, d):
    # points far apart at a small temperature: from zero potentials every
    # row's sum of 2^s underflows; forced stabilised mode has no fallback,
    # so the iteration reports GW_ENUMERIC (auto mode recovers)
    x, a, y, b = _problem(n=256, m=224, d=d, scale=3.0)
    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    with pytest.raises(L.GWError) as ei:
        ctx.solve(dev(x), dev(a), dev(y), dev(b), 0.01, 0.01, 1, 3, mode="stabilised")
    assert _code(ei) == L.GW_ENUMERIC
    r = ctx.solve(dev(x), dev(a), dev(y), dev(b), 0.01, 0.01, 1, 3, mode="auto")
    assert np.isfinite(r["loss_lift"]) and r["safe_iters"] > 0


@pytest.mark.parametrize("prec,d", [("fp32", 3), ("fp32", 32), ("bf16", 32)])
def test_stepwise_equals_whole_solve_bitwise(gw, prec, d):
    x, a, y, b = _problem(n=700, m=500, d=d, seed=9)
    X, A, Y, B = dev(x), dev(a), dev(y), dev(b)
    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    whole = ctx.solve(X, A, Y, B, 0.5, 0.05, 20, 30, precision=prec)
    ctx.solve_begin(X, A, Y, B, 0.5, 0.05, 20, 30, precision=prec)
    assert ctx.solve_advance(10) == 10
    torch.cuda.synchronize()
    # another solve on the same context in between does not disturb it
    other = ctx.solve(X, A, Y, B, 0.3, 0.3, 2, 10, precision=prec)
    assert np.isfinite(other["loss_lift"])
    assert ctx.solve_advance(7) == 17
    assert ctx.solve_advance(5) == 20  # stops at n_outer
    assert ctx.solve_advance(1) == 20
    part = ctx.solve_end()
    for k in ("loss_lift", "egw_objective", "kl", "marginal_err", "gamma_step", "safe_iters", "outer_done"):
        assert part[k] == whole[k], k
    for k in ("f", "g", "gamma"):
        assert torch.equal(part[k], whole[k]), k


def test_stepwise_state_errors(gw):
    x, a, y, b = _problem()
    ctx = gw.Context()
    ctx.set_penalty(2, "sqeuclid")
    with pytest.raises(L.GWError) as ei:
        ctx.solve_advance(1)
    assert _code(ei) == L.GW_ESTATE
    ctx.solve_begin(dev(x), dev(a), dev(y), dev(b), 0.1, 0.1, 3, 5)
    with pytest.raises(L.GWError) as ei:  # no outer step yet
        ctx.solve_end()
    assert _code(ei) == L.GW_ESTATE
    ctx.solve_begin(dev(x), dev(a), dev(y), dev(b), 0.1, 0.1, 3, 5)
    with pytest.raises(L.GWError) as ei:
        ctx.solve_advance(-1)
    assert _code(ei) == L.GW_EINVAL
    assert ctx.solve_advance(2) == 2
    r = ctx.solve_end()  # after 2 of 3 steps: the coupling after step 2
    assert r["outer_done"] == 2
    two = ctx.solve(dev(x), dev(a), dev(y), dev(b), 0.1, 0.1, 2, 5)
    assert r["loss_lift"] == two["loss_lift"]
    with pytest.raises(L.GWError) as ei:  # released by end
        ctx.solve_advance(1)
    assert _code(ei) == L.GW_ESTATE
    with pytest.raises(L.GWError) as ei:  # invalid inputs at begin
        ctx.solve_begin(dev(x), dev(a * 2), dev(y), dev(b), 0.1, 0.1, 3, 5)
    assert _code(ei) == L.GW_EINVAL


def test_warm_resume_through_public_outputs(gw):
    # 20 outer steps at one eps against 10 steps, then 10 more started from
    # the returned Gamma_10 and potentials (Algorithm 1 initialisation with
    # Gamma_0 and warm potentials, Appendix B.1): the only difference is the
    # single-precision rounding of the handed-over state
    x, a, y, b = _problem(n=600, m=520, d=3, seed=11)
    X, A, Y, B = dev(x), dev(a), dev(y), dev(b)
    ctx = gw.Context()
    ctx.set_penalty(2, "features")
    whole = ctx.solve(X, A, Y, B, 0.2, 0.2, 20, 40)
    first = ctx.solve(X, A, Y, B, 0.2, 0.2, 10, 40)
    second = ctx.solve(X, A, Y, B, 0.2, 0.2, 10, 40, gamma0=first["gamma"], f0=first["f"], g0=first["g"])
    rel = abs(second["loss_lift"] - whole["loss_lift"]) / abs(whole["loss_lift"])
    print("resume rel", rel, "gamma", float((second["gamma"] - whole["gamma"]).abs().max()))
    assert rel < 1e-5
    assert float((second["gamma"] - whole["gamma"]).abs().max()) < 1e-5 * float(whole["gamma"].abs().max()) + 1e-7
