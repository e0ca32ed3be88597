"""torch.autograd front end: J(c) with its adjoint gradient and Gauss-Newton
Hessian-vector product.

    J = WaveMisfit.apply(c, solver, wavelet, d_obs, sigma)
    g, = torch.autograd.grad(J, c, create_graph=True)     # adjoint gradient
    Hv, = torch.autograd.grad(g, c, grad_outputs=v)        # Gauss-Newton H v

The second derivative is the Gauss-Newton Hessian (J_F^T Gamma^-1 J_F, the
operator Newton-CG applies in the paper's Sec. 4), not the full Hessian:
it omits the term weighted by the data residual. All arithmetic runs in
the HIP library; the gradient is computed together with J (one forward and
one adjoint solve) and the forward history (checkpoints or autoencoder
latents) is reused by every Hv at the same c."""
from __future__ import annotations

import torch


class _Gradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, solver, g):
        ctx.solver = solver
        ctx.save_for_backward(c)
        return g.clone()

    @staticmethod
    def backward(ctx, w):
        (c,) = ctx.saved_tensors
        Hw = ctx.solver.hessvec(c.detach(), w.detach().to(torch.float32).contiguous())
        return Hw, None, None


class WaveMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, solver, wavelet, d_obs, sigma):
        J, g = solver.gradient(c.detach(), wavelet, d_obs, sigma)
        ctx.solver = solver
        ctx.save_for_backward(c, g)
        return torch.tensor(J, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, gJ):
        c, g = ctx.saved_tensors
        grad = _Gradient.apply(c, ctx.solver, g)
        return grad * gJ.to(grad.dtype), None, None, None, None
