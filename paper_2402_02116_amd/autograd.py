"""Differentiable Frechet operator and Laplacian for torch.autograd.

FrechetFn maps relative model maps q (the plan's real type, [5, nz, nx], dm_p = m0_p q_p)
to the complex receiver data J q of every system of a plan (eqs. F, YM, F0,
uY); its backward applies the adjoint (eqs. ad1, ua): for a real input and
PyTorch's conjugate-Wirtinger convention the vector-Jacobian product of an
output gradient g is m0 Re(J* g).  LaplacianFn is the periodic 5-point
Laplacian of the generalised Tikhonov term (eq. obj); it is self-adjoint.
Both run entirely in the HIP kernels of the plan.
"""

import torch


class FrechetOperator:
    """The linearisation point of one DBI step: plan, background fields u^b,
    model scales m0 (5 values) and the inner-solve tolerance."""

    def __init__(self, plan, ub, m0, rtol=1e-6, maxit=1000):
        self.plan, self.ub, self.rtol, self.maxit = plan, ub, rtol, maxit
        self.m0 = [float(v) for v in torch.as_tensor(m0).reshape(5).tolist()]


class FrechetFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, op):
        ctx.op = op
        return op.plan.frechet_rel(op.ub, q.detach().contiguous(), op.m0, op.rtol, op.maxit)

    @staticmethod
    def backward(ctx, g):
        op = ctx.op
        gq = op.plan.adjoint_rel(op.ub, g.detach().contiguous(), op.m0, op.rtol, op.maxit)
        return gq, None


class LaplacianFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, plan):
        ctx.plan = plan
        return plan.laplacian(q.detach().contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.laplacian(g.detach().contiguous()), None


def frechet(q, op):
    return FrechetFn.apply(q, op)


def tikhonov_loss(q, op, r, lam, reg="laplacian"):
    """||J q - r||^2 / ||r||^2 + lam ||L q||^2 as a differentiable torch scalar."""
    res = frechet(q, op) - r
    mis = torch.sum(res.real ** 2 + res.imag ** 2) / torch.sum(r.real ** 2 + r.imag ** 2)
    Lq = LaplacianFn.apply(q, op.plan) if reg == "laplacian" else q
    return mis + lam * torch.sum(Lq * Lq)
