"""torch.autograd.Function around the library's recorded forward and hand-written reverse
pass: u_K = MGCNNUnrolled.apply(weights, solver, a, b, f, K).

Gradients flow to the flat weight vector and to f; the coefficients a, b are inputs of the
problem and receive none.  All arithmetic runs in libmgcnn.so; this module only marshals.
"""
from __future__ import annotations

import torch


class MGCNNUnrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weights, solver, a, b, f, K: int):
        solver.set_weights_device(weights.detach().contiguous())
        solver.setup(a, b)
        u = torch.zeros_like(f)
        solver.forward(f, u, K, record=True)
        ctx.solver = solver
        ctx.f_ref = f          # the recorded forward reads f again in the reverse pass
        return u

    @staticmethod
    def backward(ctx, grad_u):
        S = ctx.solver
        df = torch.zeros_like(ctx.f_ref) if ctx.needs_input_grad[4] else None
        dw = S.backward(grad_u.contiguous(), dL_df=df)
        return dw, None, None, None, df, None


class MGCNNLoss(torch.autograd.Function):
    """L = mean_i ||f_i - A_i u_i||^2 / ||f_i||^2 with the library's operator."""

    @staticmethod
    def forward(ctx, u, solver, f):
        du = torch.empty_like(u)
        df = torch.empty_like(f)
        val = solver.loss(f, u, du, df)
        ctx.save_for_backward(du, df)
        return torch.tensor(val, dtype=torch.float64, device=u.device)

    @staticmethod
    def backward(ctx, g):
        du, df = ctx.saved_tensors
        s = g.to(torch.float32)
        return du * s, None, df * s
