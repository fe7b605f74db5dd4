"""Backward of C = A B on the GPU against the oracle: dB = A^T dC through the
packed transpose and dA = (dC B^T) on A's mask (SDDMM), in packed order."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import ops, synth
from paper_2307_03930_amd.autograd import rosko_matmul
from tests.gpu_helpers import dev, err, say

pytestmark = pytest.mark.gpu
TOL = 1e-5


def setup_module(_m):
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    O.build(force=False)


def _dA_scale(pk, dC, B):
    """|dC| |B|^T at each kept entry, packed order."""
    return O.grad_dA_packed(pk, np.abs(dC), np.abs(B))


@pytest.mark.parametrize("M,K,N,mr", [(32, 64, 16, 8), (100, 257, 190, 32), (96, 130, 1, 16),
                                      (64, 200, 700, 64), (70, 90, 2100, 32),
                                      # panels of <= 8 rows and N <= 1024: the LDS kernel
                                      (37, 300, 65, 8), (90, 128, 1024, 8), (50, 77, 1, 4),
                                      (16, 40, 300, 1), (201, 513, 257, 8), (9, 1000, 511, 5)])
def test_backward_small(M, K, N, mr):
    say(f"backward {M}x{K}x{N} mr={mr}")
    A = synth.sparse_matrix(M, K, 0.1, 700 + M)
    B = synth.dense_normal(K, N, 701 + N)
    dC = synth.dense_normal(M, N, 702)
    pk = O.pack(A, mr)
    P = ops.pack(dev(A), mr)
    Pt = ops.pack_transpose(dev(A), mr)
    dA, dB = ops.spmm_backward(P, Pt, dev(B), dev(dC))
    dB_ref = O.grad_dB(A, dC)
    dB_scale = np.abs(A).T.astype(np.float64) @ np.abs(dC).astype(np.float64)
    assert err(dB.cpu().numpy(), dB_ref, dB_scale) <= TOL
    dA_ref = O.grad_dA_packed(pk, dC, B)
    assert err(dA.cpu().numpy(), dA_ref, _dA_scale(pk, dC, B)) <= TOL


@pytest.mark.parametrize("mr", [32, 8])
def test_backward_grad_config_sampled(mr):
    """1024 x 4096 at 95% with B 4096 x 1024 and dC 1024 x 1024, full size on
    the GPU (mr 8: the panel height the analytic rule picks, and the LDS
    SDDMM); sampled rows of dB and every 97th dA entry checked."""
    say(f"backward 1024x4096x1024 s=0.95 mr={mr}")
    pr = synth.grad_problem()
    A, B, dC = pr.A, pr.B, pr.dC
    P = ops.pack(dev(A), mr)
    Pt = ops.pack_transpose(dev(A), mr)
    dA, dB = ops.spmm_backward(P, Pt, dev(B), dev(dC))
    ks = np.sort(synth.rng(703).choice(4096, 24, replace=False))
    Acols = np.ascontiguousarray(A[:, ks])
    dB_ref = O.grad_dB(Acols, dC)
    dB_scale = np.abs(Acols).T.astype(np.float64) @ np.abs(dC).astype(np.float64)
    e_dB = err(dB.cpu().numpy()[ks], dB_ref, dB_scale)
    pk = O.pack(A, mr)                  # dA is in the packed order of this panel height
    dA_ref = O.grad_dA_packed(pk, dC, B)
    sel = np.arange(0, pk.nnz, 97)
    e_dA = err(dA.cpu().numpy()[sel], dA_ref[sel], _dA_scale(pk, dC, B)[sel])
    say(f"  err dB {e_dB:.3e} dA {e_dA:.3e}")
    assert e_dB <= TOL and e_dA <= TOL


def test_autograd_function_matches_dense_reference():
    say("autograd function vs dense reference gradient")
    A = synth.sparse_matrix(64, 96, 0.2, 704)
    B = synth.dense_normal(96, 40, 705)
    G = synth.dense_normal(64, 40, 706)
    P = ops.pack(dev(A), 16)
    Pt = ops.pack_transpose(dev(A), 16)
    val = P.val.requires_grad_(True)
    Bd = dev(B).requires_grad_(True)
    C = rosko_matmul(P, Bd, Pt)
    (C * dev(G)).sum().backward()
    # dense reference gradient, FP64 on the CPU
    A64, B64, G64 = (x.astype(np.float64) for x in (A, B, G))
    dB_ref = A64.T @ G64
    dA_dense = (G64 @ B64.T) * (A != 0)
    assert np.allclose(Bd.grad.cpu().numpy(), dB_ref, rtol=1e-4, atol=1e-4)
    pk = O.pack(A, 16)
    order = []
    for p in range(pk.n_panels):
        for c in range(pk.panel_col_ptr[p], pk.panel_col_ptr[p + 1]):
            for z in range(pk.col_ptr[c], pk.col_ptr[c + 1]):
                order.append(dA_dense[p * 16 + pk.loc[z], pk.col_ind[c]])
    g = val.grad.cpu().numpy()
    assert np.allclose(g[: pk.nnz], np.array(order), rtol=1e-4, atol=1e-4)
    assert not g[pk.nnz:].any()
