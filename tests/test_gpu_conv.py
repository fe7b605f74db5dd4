"""Sparse direct convolution (no im2col) on the GPU against the oracle's
direct definition: every output element of 3x3 convolutions (stride 1,
padding 1) of pruned weights, ragged sizes, several plans and value types."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import ops, synth
from tests.gpu_helpers import DT, dev, err, say, threads

pytestmark = pytest.mark.gpu
TOL = 1e-5


def setup_module(_m):
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    O.build(force=False)


def _layer(C_out, C_in, H, W, sparsity, seed):
    A = synth.sparse_matrix(C_out, 9 * C_in, 1.0 - sparsity, seed)
    X = np.maximum(synth.rng(seed + 1).standard_normal((C_in, H, W)), 0).astype(np.float32)
    return A, X


# (panel height, plan): the library's plan and three explicit ones; two columns
# per lane exists only as a 32- or 64-row tile
MR_PLANS = [(mr, pa) for mr in (8, 16, 32) for pa in (None, (4, 4, 3), (4, 1, 1), (2, 2, 1))
            if pa is None or pa[0] != 2 or mr == 32]


@pytest.mark.parametrize("mr,plan_args", MR_PLANS)
@pytest.mark.parametrize("shape", [(6, 5, 7, 9), (32, 16, 14, 14), (4, 3, 1, 1), (3, 2, 3, 5),
                                   (40, 12, 10, 33)])
def test_conv_matches_direct_definition(shape, mr, plan_args):
    C_out, C_in, H, W = shape
    say(f"conv {shape} mr={mr} plan={plan_args}")
    A, X = _layer(C_out, C_in, H, W, 0.7, 950 + C_in + H)
    P = ops.pack(dev(A), mr)
    plan = None if plan_args is None else ops.make_plan(*plan_args)
    layer = ops.ConvLayer(P, C_in, H, W, plan)
    Yq = layer.run(dev(X))
    assert Yq.shape == (C_out, H * layer.Wq)
    Y = layer.unpad(Yq).cpu().numpy()
    ref = O.conv3x3_direct(A, X)
    scale = O.conv3x3_direct(A, X, absolute=True)
    assert err(Y, ref, scale) <= TOL
    # beta = 1 adds to the grid output
    Y0 = synth.dense_normal(C_out, H * layer.Wq, 951)
    Yb = dev(Y0)
    layer.run(dev(X), Yb, beta=1)
    got = layer.unpad(Yb).cpu().numpy()
    base = Y0.reshape(C_out, H, layer.Wq)[:, :, :W].astype(np.float64)
    assert err(got, ref + base, scale + np.abs(base)) <= TOL


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_conv_quantised_weights(dtype):
    """BF16 / FP8 weights: the records hold the decoded values and the FP8
    row scale applies in the epilogue, so the output matches the direct
    definition on the decoded weights."""
    A, X = _layer(24, 8, 12, 12, 0.8, 952)
    say(f"conv quantised {dtype}")
    P = ops.pack(dev(A), 16, dtype)
    Ad = O.unpack(O.pack(A, 16, DT[dtype])).astype(np.float32)
    layer = ops.ConvLayer(P, 8, 12, 12)
    Y = layer.unpad(layer.run(dev(X))).cpu().numpy()
    assert err(Y, O.conv3x3_direct(Ad, X), O.conv3x3_direct(Ad, X, absolute=True)) <= TOL


def test_conv_equals_im2col_product():
    """The direct route and the im2col route (SpMM on the materialised
    im2col matrix) give the same outputs to FP32 rounding."""
    A, X = _layer(32, 16, 20, 20, 0.9, 953)
    say("conv vs im2col route")
    P = ops.pack(dev(A), 16)
    layer = ops.ConvLayer(P, 16, 20, 20)
    Y = layer.unpad(layer.run(dev(X))).cpu().numpy().reshape(32, -1)
    Yc = ops.spmm(P, dev(synth.im2col_3x3(X))).cpu().numpy()
    scale = O.conv3x3_direct(A, X, absolute=True).reshape(32, -1)
    assert err(Y, Yc.astype(np.float64), scale) <= TOL


@pytest.mark.parametrize("sparsity", [0.7, 0.9, 0.99])
def test_conv_full_cnn_layer(sparsity):
    """The pruned 256 -> 256-channel layer at 56 x 56 (the im2col shape of the
    CNN benchmark), every output element against the threaded oracle, with
    the scheduler's panel height for the im2col product."""
    from paper_2307_03930_amd import sched
    A = synth.cnn_weights(sparsity)
    X = np.maximum(synth.rng(3).standard_normal((256, 56, 56)), 0).astype(np.float32)
    say(f"conv full layer s={sparsity}")
    Ad = dev(A)
    mr, _ = sched.candidate(sched.choose(Ad, 3136))
    P = ops.pack(Ad, mr)
    layer = ops.ConvLayer(P, 256, 56, 56)
    Y = layer.unpad(layer.run(dev(X))).cpu().numpy()
    t = threads()
    assert err(Y, O.conv3x3_direct(A, X, threads=t),
               O.conv3x3_direct(A, X, threads=t, absolute=True)) <= TOL


def test_conv_remap_after_repack():
    """A repack of the weight into the same buffers followed by remap() gives
    the new weight's convolution (the training-time use)."""
    A, X = _layer(16, 4, 9, 11, 0.6, 954)
    A2 = A * np.float32(-0.5)
    say("conv remap after repack")
    Ad = dev(A)
    P = ops.pack(Ad, 8)
    layer = ops.ConvLayer(P, 4, 9, 11)
    ws = torch.empty(max(ops.workspace_size(16, 36, 8), 1), dtype=torch.uint8, device="cuda")
    ops.pack_into(dev(A2), P, ws)
    ops.pack_result(P, ws)
    layer.remap()
    Y = layer.unpad(layer.run(dev(X))).cpu().numpy()
    assert err(Y, O.conv3x3_direct(A2, X), O.conv3x3_direct(A2, X, absolute=True)) <= TOL
