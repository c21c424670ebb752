"""Differentiable measurement and sparsity operators.

The measurement operator Phi = Theta G F Z (Sec. 2.1, eq:inverse) and the SARA
analysis operator Psi^dagger (Sec. 2.3) as ``torch.autograd.Function``.  All
four maps are linear, so each backward is the adjoint map (Sec. 3.3 uses the
same pairs: Re Phi^dagger for the data term, Psi for the sparsity term):

    Y = Phi X            (X real)   grad_X = Re Phi^dagger grad_Y
    X = Re Phi^dagger Y             grad_Y = Phi grad_X
    C = Psi^dagger X                grad_X = Psi grad_C
    X = Psi C                       grad_C = Psi^dagger grad_X

The backward passes call the other Function, so gradients of gradients
(Hessian-vector products of a data-fidelity loss, for instance) work too.
Every evaluation runs in the library's HIP kernels through a ``Problem``;
tensors are in the problem's precision and device.
"""
from __future__ import annotations

import torch


def _as(prob, t, complex_=False):
    dt = prob.cdtype if complex_ else prob.tdtype
    return t.to(device=prob.device, dtype=dt).contiguous()


class PhiFunction(torch.autograd.Function):
    """Y = Phi X: [L][ny][nx] real -> [sum M_l] complex (user order)."""

    @staticmethod
    def forward(ctx, prob, X):
        ctx.prob = prob
        return prob.phi(_as(prob, X))

    @staticmethod
    def backward(ctx, gY):
        return None, PhiAdjFunction.apply(ctx.prob, gY)


class PhiAdjFunction(torch.autograd.Function):
    """X = Re Phi^dagger Y: [sum M_l] complex -> [L][ny][nx] real."""

    @staticmethod
    def forward(ctx, prob, Y):
        ctx.prob = prob
        return prob.phi_adj(_as(prob, Y, complex_=True))

    @staticmethod
    def backward(ctx, gX):
        return None, PhiFunction.apply(ctx.prob, gX)


class PsiAdjFunction(torch.autograd.Function):
    """C = Psi^dagger X: [L][ny][nx] -> [D][L][ny][nx] (d = 0 Dirac, then db1..db8)."""

    @staticmethod
    def forward(ctx, prob, X):
        ctx.prob = prob
        return prob.psi_adj(_as(prob, X))

    @staticmethod
    def backward(ctx, gC):
        return None, PsiFunction.apply(ctx.prob, gC)


class PsiFunction(torch.autograd.Function):
    """X = Psi C = sum_d Psi_d C_d: [D][L][ny][nx] -> [L][ny][nx]."""

    @staticmethod
    def forward(ctx, prob, Cc):
        ctx.prob = prob
        return prob.psi(_as(prob, Cc))

    @staticmethod
    def backward(ctx, gX):
        return None, PsiAdjFunction.apply(ctx.prob, gX)


def phi(prob, X):
    return PhiFunction.apply(prob, X)


def phi_adj(prob, Y):
    return PhiAdjFunction.apply(prob, Y)


def psi_adj(prob, X):
    return PsiAdjFunction.apply(prob, X)


def psi(prob, Cc):
    return PsiFunction.apply(prob, Cc)
