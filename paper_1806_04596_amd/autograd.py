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

``l21_psi_adj`` is the l2,1 term of a loss, ||Psi^dagger X||_{2,1}, differentiated
with checkpointed per-channel recomputation: only the per-row sums of squares are
kept between forward and backward, and the coefficients are recomputed a few
channels at a time.
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


class L21PsiAdjFunction(torch.autograd.Function):
    """s = sum_r wbar_r ||(Psi^dagger X)_r||_2, the l2,1 norm of Sec. 2.3 (a row r is one
    coefficient (d, pixel) across the L channels), with checkpointed per-channel
    recomputation: the forward builds the per-row sums of squares S [D][ny][nx] (FP64)
    `chunk` channels at a time and keeps only S; the backward recomputes each chunk's
    coefficients, scales them by g wbar_r / ||row r|| (zero rows give zero, the
    subgradient of least norm) and synthesises them into that chunk of the gradient.
    Extra device memory: one chunk's coefficients [D][chunk][ny][nx] and S, instead of
    the whole [D][L][ny][nx]."""

    @staticmethod
    def forward(ctx, prob, X, wbar, chunk):
        X = _as(prob, X)
        S = torch.empty((prob.D, prob.ny, prob.nx), dtype=torch.float64, device=prob.device)
        for l0 in range(0, prob.L, chunk):
            n = min(chunk, prob.L - l0)
            prob.l21_rowsq(prob.psi_adj(X[l0:l0 + n]), S, accumulate=l0 > 0)
        wb = None if wbar is None else _as(prob, wbar)
        val = prob.l21_from_rowsq(S, wb)
        ctx.prob, ctx.chunk, ctx.wbar = prob, chunk, wb
        ctx.save_for_backward(X, S)
        return torch.tensor(val, dtype=torch.float64, device=prob.device)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g):
        X, S = ctx.saved_tensors
        prob, chunk = ctx.prob, ctx.chunk
        scale = float(g)
        grad = torch.empty_like(X)
        for l0 in range(0, prob.L, chunk):
            n = min(chunk, prob.L - l0)
            Cc = prob.l21_rowscale(prob.psi_adj(X[l0:l0 + n]), S, ctx.wbar, scale)
            prob.psi(Cc, grad[l0:l0 + n])
        return None, grad, None, None


def phi(prob, X):
    return PhiFunction.apply(prob, X)


def phi_adj(prob, Y):
    return PhiAdjFunction.apply(prob, Y)


def psi_adj(prob, X):
    return PsiAdjFunction.apply(prob, X)


def psi(prob, Cc):
    return PsiFunction.apply(prob, Cc)


def l21_psi_adj(prob, X, wbar=None, chunk=4):
    """sum_r wbar_r ||(Psi^dagger X)_r||_2 with checkpointed per-channel recomputation
    (`chunk` channels of coefficients alive at a time); differentiable in X."""
    if chunk < 1:
        raise ValueError("chunk must be >= 1")
    return L21PsiAdjFunction.apply(prob, X, wbar, int(chunk))
