"""Backward of C = A B on the GPU against the oracle: dB = A^T dC through the
packed transpose and dA = (dC B^T) on A's mask (SDDMM), in packed order."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import ops, synth
from paper_2307_03930_amd.autograd import PackedWeight, rosko_matmul
from tests.gpu_helpers import dev, err, say, threads

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
                                      (16, 40, 300, 1), (201, 513, 257, 8), (9, 1000, 511, 5),
                                      # panels of 9..16 rows, and N in 1024-column chunks
                                      # (ragged last chunk; N % 4 != 0 takes element loads)
                                      (50, 200, 700, 16), (40, 300, 2500, 16),
                                      (33, 100, 1027, 8), (20, 64, 3136, 12), (64, 96, 2049, 4),
                                      # panels of 17..32 rows: 256-column chunks
                                      (70, 300, 256, 32), (45, 130, 777, 20), (96, 64, 3136, 32)])
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
def test_backward_grad_config_full(mr):
    """1024 x 4096 at 95% with B 4096 x 1024 and dC 1024 x 1024, full size
    (mr 8: the panel height the analytic rule picks, and the LDS SDDMM);
    every element of dB and every dA entry against the threaded oracle."""
    say(f"backward 1024x4096x1024 s=0.95 mr={mr}")
    pr = synth.grad_problem()
    A, B, dC = pr.A, pr.B, pr.dC
    P = ops.pack(dev(A), mr)
    Pt = ops.pack_transpose(dev(A), mr)
    dA, dB = ops.spmm_backward(P, Pt, dev(B), dev(dC))
    t = threads()
    dB_ref = O.grad_dB(A, dC, threads=t)
    dB_scale = O.grad_dB(np.abs(A), np.abs(dC), threads=t)
    e_dB = err(dB.cpu().numpy(), dB_ref, dB_scale)
    pk = O.pack(A, mr)                  # dA is in the packed order of this panel height
    dA_ref = O.grad_dA_packed(pk, dC, B, threads=t)
    dA_scale = O.grad_dA_packed(pk, np.abs(dC), np.abs(B), threads=t)
    e_dA = err(dA.cpu().numpy(), dA_ref, dA_scale)
    say(f"  err dB {e_dB:.3e} dA {e_dA:.3e}")
    assert e_dB <= TOL and e_dA <= TOL


def _dense_grads(A, B, G):
    A64, B64, G64 = (x.astype(np.float64) for x in (A, B, G))
    return (G64 @ B64.T) * (A != 0), A64.T @ G64


def test_autograd_function_matches_dense_reference():
    """dW on W's mask (zero elsewhere) and dB against the dense FP64
    gradients, through the autograd function on the dense weight."""
    say("autograd function vs dense reference gradient")
    A = synth.sparse_matrix(64, 96, 0.2, 704)
    B = synth.dense_normal(96, 40, 705)
    G = synth.dense_normal(64, 40, 706)
    W = dev(A).requires_grad_(True)
    Bd = dev(B).requires_grad_(True)
    C = rosko_matmul(W, Bd, mr=16)
    (C * dev(G)).sum().backward()
    dW_ref, dB_ref = _dense_grads(A, B, G)
    sc_W = (np.abs(G).astype(np.float64) @ np.abs(B).T.astype(np.float64)) * (A != 0)
    assert err(W.grad.cpu().numpy(), dW_ref, sc_W) <= TOL
    assert err(Bd.grad.cpu().numpy(), dB_ref, np.abs(A).T.astype(np.float64)
               @ np.abs(G).astype(np.float64)) <= TOL
    assert not W.grad.cpu().numpy()[A == 0].any()


def test_autograd_training_steps_repack():
    """Three SGD steps on W with a magnitude prune between them: each forward
    repacks the updated W into the same buffers, and its output and
    gradients match the oracle on that step's W (the update is seen)."""
    say("autograd training steps with repacking")
    A = synth.sparse_matrix(128, 300, 0.3, 707)
    B = synth.dense_normal(300, 96, 708)
    G = synth.dense_normal(128, 96, 709)
    W = dev(A).requires_grad_(True)
    Bd, Gd = dev(B), dev(G)
    pw = PackedWeight(W.detach(), mr=16)
    for step in range(3):
        Wh = W.detach().cpu().numpy().copy()
        C = rosko_matmul(W, Bd, pw)
        (C * Gd).sum().backward()
        pw.check()
        assert err(C.detach().cpu().numpy(), O.spmm(Wh, B), O.abs_product(Wh, B)) <= TOL
        dW_ref, _ = _dense_grads(Wh, B, G)
        sc_W = (np.abs(G).astype(np.float64) @ np.abs(B).T.astype(np.float64)) * (Wh != 0)
        assert err(W.grad.cpu().numpy(), dW_ref, sc_W) <= TOL
        with torch.no_grad():
            W -= 0.01 * W.grad
            W.grad = None
            if step == 1:   # prune the 20% smallest magnitudes of the kept entries
                kept = W[W != 0].abs()
                thr = kept.kthvalue(max(1, int(0.2 * kept.numel()))).values
                W[W.abs() <= thr] = 0.0


@pytest.mark.parametrize("N", [96, 1500])
def test_backward_after_overflowed_pack_stays_in_bounds(N):
    """A repack into buffers too small for the matrix leaves pointer arrays
    that run past the capacities; the SDDMM clamps every index into them, so
    dA is written only below its capacity (a sentinel beyond survives), also
    when N is split into column chunks."""
    import ctypes as C
    from paper_2307_03930_amd import _lib as L
    say(f"backward after an overflowed pack, N={N}")
    A = synth.sparse_matrix(64, 256, 0.2, 710)
    B = synth.dense_normal(256, N, 711)
    dC = synth.dense_normal(64, N, 712)
    Ad = dev(A)
    nnz, ncols, nrec = ops.pack_query(Ad, 8)
    P = ops._alloc(64, 256, 8, L.ROSKO_F32, nnz, ncols, nrec, Ad.device)
    P.nnz, P.ncols, P.nrec = nnz // 2, ncols // 2, nrec // 2
    ws = torch.empty(ops.workspace_size(64, 256, 8), dtype=torch.uint8, device="cuda")
    ops.pack_into(Ad, P, ws)
    with pytest.raises(L.RoskoError):
        ops.pack_result(P, ws)
    P.nnz, P.ncols, P.nrec = nnz // 2, ncols // 2, nrec // 2
    dA = torch.full((nnz,), 123.0, dtype=torch.float32, device="cuda")
    st = P.struct()
    n = C.c_size_t(0)
    L.check(L.lib().rosko_spmm_backward_workspace_size(C.byref(st), None, N, C.byref(n)))
    assert (n.value > 0) == (N > 1024)
    bw = torch.empty(max(n.value, 1), dtype=torch.uint8, device="cuda")
    Bd, dCd = dev(B), dev(dC)
    L.check(L.lib().rosko_spmm_backward(
        C.byref(st), None, C.c_void_p(Bd.data_ptr()), N, C.c_void_p(dCd.data_ptr()),
        N, N, None, N, C.c_void_p(dA.data_ptr()), nnz // 2, C.c_void_p(bw.data_ptr()),
        n.value, ops._stream_ptr()))
    torch.cuda.synchronize()
    assert bool((dA[nnz // 2:] == 123.0).all())
