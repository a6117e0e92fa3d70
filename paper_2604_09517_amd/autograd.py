"""Differentiable solve X = A^-1 B as a torch.autograd.Function.

Forward: factor A and solve (FP64 LU with partial pivoting, or the
mixed-precision BF16 LU with partial pivoting + FP64 GMRES refinement).
Backward for an upstream gradient G = dL/dX: differentiating A X = B gives
A dX = dB - dA X, hence

    Lambda = A^-T G   (transposed solve reusing the forward factors),
    dL/dB  = Lambda,
    dL/dA  = -Lambda X^T   (outer-product update on the matrix cores).

Inputs and outputs are FP64 CUDA tensors; A is n x n, B is n or n x k.  The
work runs in the HIP library; torch only holds memory and the stream.
"""

from __future__ import annotations

import torch

from . import api


def _fortran_copy(t):
    if t.dim() == 1:
        return t.detach().contiguous().clone()
    out = api.fortran_empty(t.shape[0], t.shape[1], device=t.device)
    out.copy_(t.detach())
    return out


class _SolveFP64(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, nb):
        LU = _fortran_copy(A)
        _, ipiv, info = api.lu_factor(LU, nb)
        if info > 0:
            raise RuntimeError(f"solve: matrix is exactly singular (zero pivot at column {info})")
        X = _fortran_copy(B)
        api.lu_solve(LU, ipiv, X)
        ctx.save_for_backward(LU, ipiv, X)
        return X

    @staticmethod
    def backward(ctx, G):
        LU, ipiv, X = ctx.saved_tensors
        Lam = _fortran_copy(G)
        api.lu_solve(LU, ipiv, Lam, trans=True)
        n = LU.shape[0]
        dA = None
        if ctx.needs_input_grad[0]:
            dA = api.fortran_empty(n, n, device=LU.device)
            api.outer_update(dA, Lam if Lam.dim() == 2 else Lam.view(n, 1),
                             X if X.dim() == 2 else X.view(n, 1))
        dB = Lam if ctx.needs_input_grad[1] else None
        return dA, dB, None


class _SolveMixed(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, opts_kw):
        Ad = A.detach()
        if Ad.stride(0) != 1:
            Ad = _fortran_copy(Ad)
        Bd = B.detach()
        if Bd.dim() == 2 and Bd.stride(0) != 1:
            Bd = _fortran_copy(Bd)
        X, rep, work, ipiv = api.mxp_solve(Ad, Bd, **opts_kw)
        ctx.save_for_backward(Ad, work, ipiv if ipiv is not None else torch.empty(0), X)
        ctx.opts_kw = dict(opts_kw)
        ctx.report = rep
        return X

    @staticmethod
    def backward(ctx, G):
        Ad, work, ipiv, X = ctx.saved_tensors
        kw = dict(ctx.opts_kw)
        kw.update(trans=True, reuse_factors=True)
        Lam, _, _, _ = api.mxp_solve(Ad, _fortran_copy(G), work=work,
                                     ipiv=ipiv if ipiv.numel() else None, **kw)
        n = Ad.shape[0]
        dA = None
        if ctx.needs_input_grad[0]:
            dA = api.fortran_empty(n, n, device=Ad.device)
            api.outer_update(dA, Lam if Lam.dim() == 2 else Lam.view(n, 1),
                             X if X.dim() == 2 else X.view(n, 1))
        dB = Lam if ctx.needs_input_grad[1] else None
        return dA, dB, None


def solve(A, B, mode="fp64", nb=256, **mxp_kw):
    """X = A^-1 B, differentiable in A and B.

    mode "fp64": LU with partial pivoting in FP64.
    mode "bf16_ir": BF16 LU with partial pivoting on FP32 panel values and
    FP64 GMRES refinement (keyword arguments go to api.mxp_solve)."""
    if mode == "fp64":
        return _SolveFP64.apply(A, B, nb)
    if mode == "bf16_ir":
        kw = dict(prec="bf16", pivot=True, nb=nb, refine="gmres", restart=100,
                  max_outer=30, max_inner_total=1000)
        kw.update(mxp_kw)
        return _SolveMixed.apply(A, B, kw)
    raise ValueError(f"unknown mode {mode!r}")
