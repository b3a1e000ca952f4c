"""Differentiable multi-component complex solve x = A^-1 b.

The plane tensors are opaque to autograd: the gradient flowing into / out of a plane
tensor is itself a complex multi-component value in the same plane layout, with the
PyTorch complex convention grad = dL/dRe + i dL/dIm.  For x = A^-1 b:

    g_b = A^-H g_x          (conjugate-transpose solve reusing the saved LU factors)
    g_A = -g_b x^H          (rank-nrhs update)

both computed by the library (mplu_zgetrs with trans 'C', then mplu_zgemm with
opB 'C' and alpha = -1); nothing is recomputed or evaluated in torch.
"""
from __future__ import annotations

import torch


class MPSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, panel=64, method="3m"):
        from . import gesv

        LU = A.detach().clone()
        X = B.detach().clone()
        ipiv, info = gesv(LU, X, panel=panel, method=method)
        ctx.save_for_backward(LU, ipiv, X)
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, gX):
        from . import gemm, getrs

        LU, ipiv, X = ctx.saved_tensors
        gB = gX.detach().to(torch.float64).contiguous().clone()
        getrs(LU, ipiv, gB, trans="C")
        gA = None
        if ctx.needs_input_grad[0]:
            gA = gemm(gB, X, None, opA="N", opB="C", alpha=-1, method="4m")
        return gA, (gB if ctx.needs_input_grad[1] else None), None, None


def solve(A: torch.Tensor, B: torch.Tensor, panel: int = 64, method="3m",
          check_errors: bool = False) -> torch.Tensor:
    """X = A^-1 B on plane tensors, differentiable in A and B.  With check_errors, an
    exactly singular A (a zero pivot, info > 0) raises torch.linalg.LinAlgError after the
    one synchronisation that reading info takes."""
    if torch.is_grad_enabled() and (A.requires_grad or B.requires_grad):
        X = MPSolve.apply(A, B, panel, method)
        info = X.grad_fn.info
    else:
        from . import gesv

        X = B.detach().clone()
        _, info = gesv(A.detach().clone(), X, panel=panel, method=method)
    if check_errors:
        k = int(info.item())
        if k > 0:
            raise torch.linalg.LinAlgError(f"exactly singular: zero pivot in column {k}")
    return X


def lu_factor(A: torch.Tensor, panel: int = 64, method="3m"):
    """(LU, piv, info) of a plane tensor A, which is left unchanged (torch.linalg
    lu_factor style: piv is 1-based, LAPACK order)."""
    from . import getrf

    LU = A.detach().clone()
    piv, info = getrf(LU, panel=panel, method=method)
    return LU, piv, info


def lu_solve(LU: torch.Tensor, piv: torch.Tensor, B: torch.Tensor,
             adjoint: bool = False) -> torch.Tensor:
    """X = A^-1 B (or A^-H B with adjoint) from lu_factor's output; B is left unchanged."""
    from . import getrs

    X = B.detach().clone()
    return getrs(LU, piv, X, trans="C" if adjoint else "N")
