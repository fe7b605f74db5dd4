"""torch.autograd.Function over the Rosko SpMM.

Forward  C = A B with A packed (Alg. 2).
Backward dB = A^T dC as a Rosko SpMM over the packed transpose of A, and
         dA = (dC B^T) on A's kept entries only, in packed order (SDDMM), so
         pruned weights receive no gradient.  This follows the training
         decomposition of Sec. 5.4 (forward and activation gradient as
         sparse products), with the weight gradient restricted to the mask.

The trainable tensor is the packed value buffer `P.val` (FP32 values); its
spare entries past nnz get zero gradient.  Pt must pack the same matrix.
"""
from __future__ import annotations

import torch

from . import ops


class RoskoSpMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val: torch.Tensor, B: torch.Tensor, P: ops.PackedMatrix,
                Pt: ops.PackedMatrix | None):
        if val.data_ptr() != P.val.data_ptr():
            raise ValueError("val must be the packed value buffer P.val")
        ctx.P, ctx.Pt = P, Pt
        ctx.save_for_backward(B)
        return ops.spmm(P, B)

    @staticmethod
    def backward(ctx, dC: torch.Tensor):
        (B,) = ctx.saved_tensors
        P, Pt = ctx.P, ctx.Pt
        need_dA, need_dB = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if need_dB and Pt is None:
            raise ValueError("dB needs the packed transpose Pt")
        dA, dB = ops.spmm_backward(P, Pt if need_dB else None, B, dC.contiguous(),
                                   need_dB=need_dB, need_dA=need_dA)
        gval = None
        if need_dA:
            gval = torch.zeros_like(P.val)
            gval[: P.nnz] = dA
        return gval, dB, None, None


def rosko_matmul(P: ops.PackedMatrix, B: torch.Tensor, Pt: ops.PackedMatrix | None = None):
    return RoskoSpMM.apply(P.val, B, P, Pt)
