"""Pruned training with on-the-fly repacking: every product of every step
against the FP64 oracle on that step's weights and inputs, across magnitude
pruning rounds (the training decomposition of Sec. 5.4)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import synth, training
from tests.gpu_helpers import dev, err, say

pytestmark = pytest.mark.gpu
TOL = 1e-5


def setup_module(_m):
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    O.build(force=False)


def _sddmm_ref(dC, Bt, mask):
    """(dC B^T) on the mask, FP64, and its |.| scale."""
    d64, b64 = dC.astype(np.float64), Bt.astype(np.float64)
    return (d64 @ b64.T) * mask, (np.abs(d64) @ np.abs(b64).T) * mask


@pytest.mark.parametrize("mr", [8, 16])
def test_pruned_chain_steps_match_oracle(mr):
    """Six SGD steps of the two-layer chain (3x3 convolution 32 -> 64
    channels on 14 x 14 im2col activations, then a 1x1 convolution 64 -> 64),
    pruned from 50% to 80% sparsity in rounds of 10% of the weights: each
    step's C1, C2, dH = W2^T dC2 and the masked weight gradients against the
    oracle on that step's weights; pruned weights stay zero and get no
    gradient; the loss falls."""
    g = synth.rng(720)
    K1, M, N = 32 * 9, 64, 14 * 14
    W1 = (g.standard_normal((M, K1)) * 0.05).astype(np.float32)
    W2 = (g.standard_normal((M, M)) * 0.1).astype(np.float32)
    training.magnitude_prune(torch.from_numpy(W1), 0.5)
    training.magnitude_prune(torch.from_numpy(W2), 0.5)
    X = np.maximum(synth.dense_normal(K1, N, 721), 0.0).astype(np.float32)
    T = synth.dense_normal(M, N, 722)
    chain = training.PrunedChain(dev(W1), dev(W2), mr)
    Xd, Td = dev(X), dev(T)
    losses = []
    for step in range(6):
        s = training.schedule(step, 2, 0.1, 0.8, 0.5)
        chain.prune(s)
        W1h = chain.W1.detach().cpu().numpy().copy()
        W2h = chain.W2.detach().cpu().numpy().copy()
        say(f"chain step {step}: sparsity {s:.2f}, nnz {np.count_nonzero(W1h)} + "
            f"{np.count_nonzero(W2h)}")
        C1, H, C2 = chain.forward(Xd)
        for t in (C1, H, C2):
            t.retain_grad()
        loss = ((C2 - Td) ** 2).mean()
        loss.backward()
        chain.pw1.check()
        chain.pw2.check()
        c1, h, c2 = (x.detach().cpu().numpy() for x in (C1, H, C2))
        assert err(c1, O.spmm(W1h, X), O.abs_product(W1h, X)) <= TOL
        assert err(c2, O.spmm(W2h, h), O.abs_product(W2h, h)) <= TOL
        dC2 = C2.grad.cpu().numpy()
        dH = H.grad.cpu().numpy()
        dC1 = C1.grad.cpu().numpy()
        assert err(dH, O.grad_dB(W2h, dC2), O.grad_dB(np.abs(W2h), np.abs(dC2))) <= TOL
        for Wh, grad, dC, Bin in ((W2h, chain.W2.grad, dC2, h), (W1h, chain.W1.grad, dC1, X)):
            mask = Wh != 0
            ref, sc = _sddmm_ref(dC, Bin, mask)
            got = grad.cpu().numpy()
            assert err(got, ref, sc) <= TOL
            assert not got[~mask].any()
        losses.append(float(loss.detach()))
        with torch.no_grad():
            for W in (chain.W1, chain.W2):
                W -= 0.5 * W.grad
                W.grad = None
        assert not chain.W1.detach().cpu().numpy()[W1h == 0].any()
    say(f"losses {[round(x, 4) for x in losses]}")
    assert losses[-1] < losses[0]
