"""torch.autograd front end of the MAP objective (paper Sec. 2): the data misfit
J(c) with its adjoint gradient and Hessian-vector products, and the BiLaplacian
prior term R(c).

    J = WaveMisfit.apply(c, solver, wavelet, d_obs, sigma)        # Gauss-Newton second derivative
    J = WaveMisfit.apply(c, solver, wavelet, d_obs, sigma, False)  # full-Newton second derivative
    R = BiLaplacianPrior.apply(c, solver)                          # prior set by solver.set_prior
    g, = torch.autograd.grad(J + R, c, create_graph=True)          # adjoint gradient + prior gradient
    Hv, = torch.autograd.grad(g, c, grad_outputs=v)                # Hessian action

By default the misfit's second derivative is the Gauss-Newton Hessian
(J_F^T Gamma^-1 J_F, the operator Newton-CG applies in the paper's Sec. 4),
which omits the term weighted by the data residual. Passing False selects the
full-Newton product, which needs a full, autoencoder or time store. The prior's is exact
(dx^dims A A). All arithmetic runs in the HIP library. The gradient is computed
together with J (one forward and one adjoint solve), and the forward history
(checkpoints or autoencoder latents) is reused by every Hv at the same c."""
from __future__ import annotations

import torch


class _Gradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, solver, g, gauss_newton):
        ctx.solver = solver
        ctx.gauss_newton = gauss_newton
        ctx.save_for_backward(c)
        return g.clone()

    @staticmethod
    def backward(ctx, w):
        (c,) = ctx.saved_tensors
        Hw = ctx.solver.hessvec(c.detach(), w.detach().to(torch.float32).contiguous(), ctx.gauss_newton)
        return Hw, None, None, None


class WaveMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, solver, wavelet, d_obs, sigma, gauss_newton=True):
        J, g = solver.gradient(c.detach(), wavelet, d_obs, sigma)
        ctx.solver = solver
        ctx.gauss_newton = bool(gauss_newton)
        ctx.save_for_backward(c, g)
        return torch.tensor(J, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, gJ):
        c, g = ctx.saved_tensors
        grad = _Gradient.apply(c, ctx.solver, g, ctx.gauss_newton)
        return grad * gJ.to(grad.dtype), None, None, None, None, None


class _PriorGradient(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, solver, g):
        ctx.solver = solver
        return g.clone()

    @staticmethod
    def backward(ctx, w):
        return ctx.solver.prior_hessvec(w.detach().to(torch.float32).contiguous()), None, None


class BiLaplacianPrior(torch.autograd.Function):
    """R(c) = 1/2 dx^dims |A (c - c0)|^2 with the prior of solver.set_prior."""

    @staticmethod
    def forward(ctx, c, solver):
        R, g = solver.prior(c.detach())
        ctx.solver = solver
        ctx.save_for_backward(c, g)
        return torch.tensor(R, dtype=torch.float64, device=c.device)

    @staticmethod
    def backward(ctx, gR):
        c, g = ctx.saved_tensors
        grad = _PriorGradient.apply(c, ctx.solver, g)
        return grad * gR.to(grad.dtype), None
