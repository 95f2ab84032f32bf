"""GW_eps as a differentiable PyTorch function.

The value is Algorithm 1's entropic GW objective (the lifted loss of
Lemma C.1 plus eps * KL of the final coupling).  Its gradients are the
envelope gradients of Appendix B.6 computed by the library's backward kernels
in the same call (the optimum is held fixed, so no gradient flows through the
Sinkhorn iterations); ``backward`` only scales them by the incoming gradient.

Weight gradients are the tangent part on the probability simplex: they satisfy
sum_i a_i g_i = 0, since adding a constant to a potential does not change the
objective along directions that keep sum(a) = 1.
"""
from __future__ import annotations

import torch

from .api import Context


class GWLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, a, y, b, gw_context: Context, params: dict):
        need = ctx.needs_input_grad[:4]
        want = tuple(k for k, nd in zip(("x", "a", "y", "b"), need) if nd)
        out = gw_context.loss_and_grad(x.detach(), a.detach(), y.detach(), b.detach(), want=want, **params)
        grads = [out["grad_" + k] for k in ("x", "a", "y", "b")]
        ctx.has = [g is not None for g in grads]
        ctx.save_for_backward(*[g if g is not None else torch.empty(0, device=x.device) for g in grads])
        ctx.result = {k: v for k, v in out.items() if not k.startswith("grad_")}
        return torch.tensor(out["egw_objective"], dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, grad_out):
        saved = ctx.saved_tensors
        go = grad_out.to(torch.float32)
        res = [s * go if h else None for s, h in zip(saved, ctx.has)]
        return res[0], res[1], res[2], res[3], None, None


def gw_loss(x, a, y, b, context: Context | None = None, **params) -> torch.Tensor:
    """Differentiable GW_eps(x, a; y, b).  ``params`` are those of
    ``Context.loss_and_grad`` (eps_start, eps_end, n_outer, n_inner,
    symmetric, precision, mode, gamma0).  The penalty of each side is the
    context's (default: squared Euclidean)."""
    ctx = context if context is not None else Context(x.device.index or 0)
    return GWLoss.apply(x, a, y, b, ctx, params)
