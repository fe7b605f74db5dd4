"""Pruned training with on-the-fly repacking (the training use of Sec. 5.4).

A two-layer chain of convolution layers written as GEMMs, as in a pruned
CNN: layer 1 is a 3x3 convolution with 256 input and 256 output channels
(weights W1, 256 x 2304, times the im2col activations X, 2304 x N), then a
ReLU, then a 1x1 convolution (W2, 256 x 256).  The loss is the mean squared
distance of the output to a target.  Both weight matrices are kept dense
with zeros at pruned positions; iterative magnitude pruning removes a fixed
fraction of the original weights every `prune_every` steps until the target
sparsity is reached (the training schedule of Sec. 5.4, read as a fraction
of the original weights per round).

Every step packs both weights and their transposes afresh (Alg. 1, on the
GPU, into buffers sized at the first pack; the four packs in one batched
call) and runs every product of the step through the library:
  forward   C1 = W1 X,  H = relu(C1),  C2 = W2 H           (Rosko SpMM, Alg. 2)
  backward  dW2 = (dC2 H^T) on W2's mask                   (SDDMM, scattered)
            dH  = W2^T dC2                                 (SpMM on the packed W2^T)
            dW1 = (dC1 X^T) on W1's mask, dC1 = dH * [C1 > 0]
The loss, the ReLU and the SGD update are the training harness around the
method (torch element-wise operations on the caller's tensors).
"""
from __future__ import annotations

import torch

from .autograd import PackedWeight, repack_weights, rosko_matmul


def magnitude_prune(W: torch.Tensor, sparsity: float) -> None:
    """Zeroes the smallest-magnitude entries of W in place so that at least
    round(sparsity * W.numel()) entries are zero (ties by position)."""
    n = W.numel()
    k = int(round(sparsity * n))
    if k <= 0:
        return
    flat = W.view(-1)
    order = torch.argsort(flat.abs(), stable=True)
    flat[order[:k]] = 0.0


class PrunedChain:
    """Weights, their packed buffers and one SGD step of the chain."""

    def __init__(self, W1: torch.Tensor, W2: torch.Tensor, mr: int = 8):
        self.W1 = W1.detach().clone().requires_grad_(True)
        self.W2 = W2.detach().clone().requires_grad_(True)
        self.pw1 = PackedWeight(self.W1.detach(), mr)
        self.pw2 = PackedWeight(self.W2.detach(), mr)

    def forward(self, X: torch.Tensor):
        # both weights and their transposes re-packed in one batched call
        repack_weights([(self.W1, self.pw1), (self.W2, self.pw2)])
        C1 = rosko_matmul(self.W1, X, self.pw1, repack=False)
        H = torch.relu(C1)
        C2 = rosko_matmul(self.W2, H, self.pw2, repack=False)
        return C1, H, C2

    def step(self, X: torch.Tensor, T: torch.Tensor, lr: float) -> torch.Tensor:
        """One SGD step; returns the loss (a device scalar)."""
        _, _, C2 = self.forward(X)
        loss = ((C2 - T) ** 2).mean()
        loss.backward()
        with torch.no_grad():
            self.W1 -= lr * self.W1.grad
            self.W2 -= lr * self.W2.grad
            self.W1.grad = None
            self.W2.grad = None
        return loss.detach()

    def prune(self, sparsity: float) -> None:
        with torch.no_grad():
            magnitude_prune(self.W1, sparsity)
            magnitude_prune(self.W2, sparsity)


def schedule(step: int, prune_every: int, per_round: float, target: float,
             start: float = 0.0) -> float:
    """Sparsity after `step` steps: `per_round` of the original weights are
    removed every `prune_every` steps, from `start` up to `target`."""
    return min(target, start + per_round * (step // prune_every))
