"""torch.autograd.Function over the efunc C ABI.

Forward = efunc_eval (Alg. 1; saves O and the log-denominator), backward =
efunc_grad (Alg. 2 / Sec. 3.6 closed forms) accumulating dL/dtheta, plus
dL/dq from the query gradient of Eq. func-normal when the queries require a
gradient.  Nothing is materialised per key-query pair; the saved state is
O and lse (2 floats per query).
"""
from __future__ import annotations

import torch

from .efunc import Engine


class EfuncFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, q: torch.Tensor, engine: Engine):
        theta_c = theta.detach().contiguous()
        q_c = q.detach().contiguous()
        want_q = q.requires_grad
        O, lse, dq, _ = engine.eval(theta_c, q_c, with_lse=True, with_qgrad=want_q)
        ctx.engine = engine
        ctx.save_for_backward(theta_c, q_c, O, lse, dq if want_q else torch.empty(0, device=q.device))
        ctx.want_q = want_q
        return O

    @staticmethod
    def backward(ctx, gO: torch.Tensor):
        theta, q, O, lse, dq = ctx.saved_tensors
        g = gO.detach().contiguous().to(torch.float32)
        gtheta = None
        if ctx.needs_input_grad[0]:
            gtheta = torch.zeros_like(theta)
            ctx.engine.grad(theta, q, O, lse, g, gtheta)
        gq = g[:, None] * dq if ctx.want_q and ctx.needs_input_grad[1] else None
        return gtheta, gq, None


def efunc_apply(theta: torch.Tensor, q: torch.Tensor, engine: Engine) -> torch.Tensor:
    """O(q) for all queries, differentiable in theta (and q)."""
    return EfuncFunction.apply(theta, q, engine)
