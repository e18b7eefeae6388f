"""Differentiable perturbation-induced solve: torch.autograd.Function over the C ABI.

Forward (Alg. 1 steps 1-4): factor the K perturbed systems A + eps_k D of every
Jacobian without pivoting, solve with B, and combine x_hat = sum_k c_k x_k.

Backward reuses the same perturbed factors transposed.  For a loss L with
upstream gradient W = dL/dx_hat:
    lambda_k = (A + eps_k D)^{-T} W
    dL/dB    = sum_k c_k lambda_k
    dL/dA_ij = - sum_k c_k sum_r lambda_k[i, r] x_k[j, r]   on the pattern of A
This is the exact gradient of x_hat (the Neumann series of Sec. II-B applied
to A^T with the same weights makes it match the gradient of x* = A^{-1} B up
to the same truncation order).
"""
from __future__ import annotations

import torch

from . import psp


class PerturbedSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, B, plan, eps, path="auto", d=None):
        squeeze = B.dim() == 2
        B3 = B.unsqueeze(-1) if squeeze else B
        F = psp.Factors(plan, values.detach().contiguous(), eps, path=path, d=d, nrhs_cap=B3.shape[2])
        Xk = F.solve(B3.detach().contiguous())
        X = F.combine(Xk)
        ctx.F = F
        ctx.squeeze = squeeze
        ctx.save_for_backward(Xk)
        return X.squeeze(-1) if squeeze else X

    @staticmethod
    def backward(ctx, gX):
        (Xk,) = ctx.saved_tensors
        F = ctx.F
        G = gX.unsqueeze(-1) if ctx.squeeze else gX
        Lk = F.solve(G.contiguous(), transpose=True)
        gB = F.combine(Lk)
        gA = F.grad_values(Lk, Xk) if ctx.needs_input_grad[0] else None
        if ctx.squeeze:
            gB = gB.squeeze(-1)
        return gA, gB if ctx.needs_input_grad[1] else None, None, None, None, None


def perturbed_solve(values, B, plan, eps, path="auto", d=None):
    """x_hat = sum_k c_k (A + eps_k D)^{-1} B, differentiable in values and B."""
    return PerturbedSolve.apply(values, B, plan, eps, path, d)
