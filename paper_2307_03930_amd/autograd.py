"""torch.autograd.Function over the Rosko SpMM, for training pruned weights.

The trainable tensor is the dense weight W (M x K, FP32, zeros at pruned
positions): the form a training loop keeps and updates.  Every forward
packs W afresh (on-the-fly packing, Sec. 4.1; the repacking that training
with Rosko pays every step, Sec. 5.4), so an optimizer step on W is seen by
the next forward.  Packing reads W's current values, so the stored
structure is W's mask at that step.

Forward  C = W B, a Rosko SpMM over the packed W (Alg. 2).
Backward dB = W^T dC, a Rosko SpMM over the packed transpose of W, and
         dW = (dC B^T) on W's kept entries only (an SDDMM in packed order,
         scattered back to W's dense layout), so pruned weights get no
         gradient.  This is the training decomposition of Sec. 5.4 with the
         weight gradient restricted to the mask.

`PackedWeight` holds the packed buffers of one weight and repacks into them
without a host synchronisation (the capacities come from the first pack;
pruning only removes entries, so later masks fit).
"""
from __future__ import annotations

import torch

from . import ops


class PackedWeight:
    """Packed buffers of a dense weight W and of W^T, refilled in place."""

    def __init__(self, W: torch.Tensor, mr: int = 16, mr_t: int | None = None):
        self.mr, self.mr_t = mr, (mr_t or mr)
        self.P = ops.pack(W, self.mr)
        self.Pt = ops.pack_transpose(W, self.mr_t)
        M, K = W.shape
        dev = W.device
        self.ws = torch.empty(max(ops.workspace_size(M, K, self.mr), 1), dtype=torch.uint8,
                              device=dev)
        self.ws_t = torch.empty(max(ops.workspace_size(M, K, self.mr_t, transpose=True), 1),
                                dtype=torch.uint8, device=dev)

    def repack(self, W: torch.Tensor) -> None:
        """Packs W (same shape; no more kept entries than the first pack) into
        the existing buffers, asynchronously."""
        ops.pack_into(W, self.P, self.ws)
        ops.pack_transpose_into(W, self.Pt, self.ws_t)

    def check(self) -> None:
        """Synchronises; raises if a repack overflowed the capacities."""
        ops.pack_result(self.P, self.ws)
        ops.pack_result(self.Pt, self.ws_t, transpose=True)


def repack_weights(pairs) -> None:
    """Re-packs several weights, each W and W^T into its PackedWeight's
    buffers, in one batched call (rosko_pack_batch: the single passes of one
    kernel form share a launch); asynchronous.  pairs: (W, PackedWeight)."""
    items = []
    for W, pw in pairs:
        Wd = W.detach()
        items.append((Wd, pw.P, pw.ws))
        items.append((Wd, pw.Pt, pw.ws_t, True))
    ops.pack_batch_into(items)


class RoskoSparseMatmul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, W: torch.Tensor, B: torch.Tensor, pw: PackedWeight, repack: bool):
        if repack:
            pw.repack(W.detach())
        ctx.pw = pw
        ctx.save_for_backward(W, B)
        return ops.spmm(pw.P, B)

    @staticmethod
    def backward(ctx, dC: torch.Tensor):
        W, B = ctx.saved_tensors
        pw = ctx.pw
        need_dW, need_dB = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dA, dB = ops.spmm_backward(pw.P, pw.Pt if need_dB else None, B, dC.contiguous(),
                                   need_dB=need_dB, need_dA=need_dW)
        dW = None
        if need_dW:
            dW = torch.zeros_like(W)
            ops.scatter_dense(pw.P, dA, dW)
        return dW, dB, None, None


def rosko_matmul(W: torch.Tensor, B: torch.Tensor, pw: PackedWeight | None = None,
                 mr: int = 16, repack: bool = True) -> torch.Tensor:
    """C = W B through the packed W; W and B receive gradients.  With `pw`
    given, W is repacked into its buffers (unless repack is False, for a W
    unchanged since the last pack); otherwise it is packed here."""
    if pw is None:
        pw = PackedWeight(W.detach(), mr)
        repack = False
    return RoskoSparseMatmul.apply(W, B, pw, repack)
