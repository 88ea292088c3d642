"""torch.autograd.Function wrappers: gradients of the PSFD solution and of the
PSFD residual loss with respect to the absorber permittivity and the field.

Forward and backward both run in the library (psfd_solve, adjoint psfd_solve,
psfd_residual, psfd_adjoint, psfd_eps_grad); only the chain-rule scalars are
applied here.  Complex gradients follow the PyTorch convention
(grad = dL/dRe + i dL/dIm).

* ``scattered_field(eps, cfg)`` -> E solving A(eps) E = b(eps).  Backward:
  mu = A^-H g, dL/d eps = k0^2 sum_alpha mu_alpha conj(Psi_alpha(E)) with
  Psi = E + R_ml[E] + E_bg on absorber rows (the field d_eps multiplies).
* ``residual_loss(E, eps, cfg)`` -> (1/N) ||A E - b||^2, N = nx ny nz (the
  residual term of the paper's physics loss).  Backward: dJ/dE = -(2/N) A^H r,
  dJ/d eps = (2 k0^2/N) sum_alpha r_alpha conj(Psi_alpha(E)), r = b - A E.
* ``pino_loss(E, eps, cfg, w0, eta_hf, lambda_hf)`` -> the whole physics loss
  with the high-frequency penalty (psfd_pino_loss).  Backward: with
  g = (1/N) r + lambda_hf H r (H = F3^-1 w^2 F3, r = b - A E),
  dJ/dE = -2 A^H g and dJ/d eps = 2 k0^2 sum_alpha g_alpha conj(Psi_alpha(E)).
"""

import torch

from .psfd import PSFD_C128, Plan


class _ScatteredField(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps, cfg, prec, tol, maxit):
        plan = Plan(cfg, eps.detach().contiguous(), prec)
        E, info = plan.solve(tol=tol, maxit=maxit)
        ctx.plan, ctx.tol, ctx.maxit = plan, tol, maxit
        ctx.save_for_backward(E)
        return E

    @staticmethod
    def backward(ctx, gE):
        (E,) = ctx.saved_tensors
        plan = ctx.plan
        mu, _ = plan.solve(b=gE.contiguous(), tol=ctx.tol, maxit=ctx.maxit, adjoint=True)
        grad = plan.eps_grad(E, mu, plan.k0 ** 2)
        plan.close()
        return grad, None, None, None, None


def scattered_field(eps, cfg, prec=PSFD_C128, tol=1e-10, maxit=20000):
    """Solve the PSFD system for permittivity `eps` (nz_abs, ny, nx) complex128 (differentiable)."""
    return _ScatteredField.apply(eps, cfg, prec, tol, maxit)


class _ResidualLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, eps, cfg):
        plan = Plan(cfg, eps.detach().contiguous())
        r, rr = plan.residual(E.detach().contiguous())
        n = cfg["nx"] * cfg["ny"] * plan.nz
        ctx.plan, ctx.n = plan, n
        ctx.save_for_backward(E, r)
        return torch.tensor(rr / n, dtype=torch.float64, device=E.device)

    @staticmethod
    def backward(ctx, gJ):
        E, r = ctx.saved_tensors
        plan, n = ctx.plan, ctx.n
        g = float(gJ)
        grad_E = plan.adjoint(r).mul_(-2.0 * g / n)
        grad_eps = plan.eps_grad(E.detach().contiguous(), r, 2.0 * plan.k0 ** 2 * g / n)
        plan.close()
        return grad_E, grad_eps, None


def residual_loss(E, eps, cfg):
    """(1/N) ||A(eps) E - b(eps)||^2 (differentiable in E and eps)."""
    return _ResidualLoss.apply(E, eps, cfg)


class _PinoLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, eps, cfg, w0, eta, lam):
        plan = Plan(cfg, eps.detach().contiguous())
        Ed = E.detach().contiguous()
        (J, _, _), g = plan.pino_loss(Ed, w0, eta, lam, grad=True)
        ctx.plan = plan
        ctx.save_for_backward(Ed, g)
        return torch.tensor(J, dtype=torch.float64, device=E.device)

    @staticmethod
    def backward(ctx, gJ):
        E, g = ctx.saved_tensors
        plan = ctx.plan
        s = float(gJ)
        grad_E = plan.adjoint(g).mul_(-2.0 * s)
        grad_eps = plan.eps_grad(E, g, 2.0 * plan.k0 ** 2 * s)
        plan.close()
        return grad_E, grad_eps, None, None, None, None


def pino_loss(E, eps, cfg, w0=1.0, eta_hf=0.0, lambda_hf=0.0):
    """The paper's physics loss (equation loss): (1/N) ||r||^2 + (lambda_hf/N) ||w F3 r||^2,
    r = A(eps) E - b(eps), w = w0 + eta_hf |nu| (differentiable in E and eps)."""
    return _PinoLoss.apply(E, eps, cfg, w0, eta_hf, lambda_hf)
