"""rosko_spmm_noalloc (no device allocation; K-split partials in the
library's own scratch) against rosko_spmm with a caller workspace: the same
bits and the oracle's FP32 bar, on two calls in a row, the second smaller."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import _lib as L
from paper_2307_03930_amd import ops, synth
from tests.gpu_helpers import dev, err, say

pytestmark = pytest.mark.gpu
TOL = 1e-5


def setup_module(_m):
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    O.build(force=False)


def _noalloc(P, B, C_out, beta, plan):
    st = P.struct()
    L.check(L.lib().rosko_spmm_noalloc(C.byref(st), ops._ptr(B), L.ROSKO_F32, B.shape[1],
                                       B.stride(0), ops._ptr(C_out), C_out.stride(0), beta,
                                       C.byref(plan) if plan is not None else None,
                                       ops._stream_ptr()))
    return C_out


def test_noalloc_matches_workspace_entry_point_twice():
    cases = [
        # (A, B, mr, plan): the 256 x 2304 x 3136 layer at 90% with 6 K splits
        # (19 MB of partials), then a smaller ragged problem with 3
        (synth.cnn_layer(0.90).A, synth.cnn_layer(0.90).B, 16, ops.make_plan(4, 4, 6)),
        (synth.sparse_matrix(77, 1031, 0.15, 900), synth.dense_normal(1031, 190, 901), 8,
         ops.make_plan(4, 2, 3)),
    ]
    for A, B, mr, plan in cases:
        say(f"noalloc {A.shape[0]}x{A.shape[1]}x{B.shape[1]} mr={mr} k_split={plan.k_split}")
        P = ops.pack(dev(A), mr)
        Bd = dev(B)
        c_ws = ops.spmm(P, Bd, plan=plan).cpu().numpy()
        Cd = torch.full((A.shape[0], B.shape[1]), 7.0, dtype=torch.float32, device="cuda")
        c_na = _noalloc(P, Bd, Cd, 0, plan).cpu().numpy()
        assert c_na.tobytes() == c_ws.tobytes()
        assert err(c_na, O.spmm(A, B, threads=8), O.abs_product(A, B, threads=8)) <= TOL
        # the automatic plan (splits capped to the scratch) and beta = 1
        C0 = synth.dense_normal(A.shape[0], B.shape[1], 902)
        Cd = dev(C0)
        got = _noalloc(P, Bd, Cd, 1, None).cpu().numpy()
        ref = O.spmm(A, B, threads=8) + C0.astype(np.float64)
        assert err(got, ref, O.abs_product(A, B, threads=8) + np.abs(C0)) <= TOL


def test_noalloc_refuses_what_does_not_fit():
    """Checked on the host before any work: a plan whose partials exceed the
    scratch, and the dense path."""
    A = synth.sparse_matrix(64, 64, 0.2, 903)
    P = ops.pack(dev(A), 16)
    st = P.struct()
    st.M = 4096                        # only the shape is read by the check
    st.n_panels = 256
    big = ops.make_plan(4, 4, 64)
    fake = C.c_void_p(0x1000)
    rc = L.lib().rosko_spmm_noalloc(C.byref(st), fake, L.ROSKO_F32, 4096, 4096, fake, 4096, 0,
                                    C.byref(big), ops._stream_ptr())
    assert rc == L.ROSKO_ESMALLBUF
    st = P.struct()
    rc = L.lib().rosko_spmm_noalloc(C.byref(st), fake, L.ROSKO_F32, 64, 64, fake, 64, 0,
                                    C.byref(ops.dense_plan()), ops._stream_ptr())
    assert rc == L.ROSKO_EUNSUPPORTED
