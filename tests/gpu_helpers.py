"""Shared helpers of the GPU parity tests (HIP path through the C ABI versus
the CPU oracle)."""
import functools
import sys

import numpy as np
import torch

import oracle as O
from paper_2307_03930_amd import ops

DT = {"f32": O.F32, "bf16": O.BF16, "fp8": O.FP8}


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def packed_to_np(P: ops.PackedMatrix) -> dict:
    torch.cuda.synchronize()
    out = {
        "panel_nz_ptr": P.panel_nz_ptr.cpu().numpy(),
        "panel_col_ptr": P.panel_col_ptr.cpu().numpy(),
        "col_ind": P.col_ind[: P.ncols].cpu().numpy(),
        "col_nnz": P.col_nnz[: P.ncols].cpu().numpy(),
        "col_ptr": P.col_ptr[: P.ncols + 1].cpu().numpy(),
        "loc": P.loc[: P.nnz].cpu().numpy(),
        "val": P.val[: P.nnz].cpu().numpy(),
        "kblk_ptr": P.kblk_ptr[: P.n_panels * ((P.K + 127) // 128 + 1)].cpu().numpy(),
        "rec": P.rec[: P.nrec].cpu().numpy().view(np.uint32),
    }
    if P.row_scale is not None:
        out["row_scale"] = P.row_scale[: P.M].cpu().numpy()
    return out


def assert_pack_equal(P: ops.PackedMatrix, ref: O.Packed) -> None:
    g = packed_to_np(P)
    assert P.nnz == ref.nnz and P.ncols == ref.ncols
    assert np.array_equal(g["panel_nz_ptr"], ref.panel_nz_ptr)
    assert np.array_equal(g["panel_col_ptr"], ref.panel_col_ptr)
    assert np.array_equal(g["col_ind"], ref.col_ind)
    assert np.array_equal(g["col_nnz"], ref.col_nnz)
    assert np.array_equal(g["col_ptr"], ref.col_ptr)
    assert np.array_equal(g["loc"], ref.loc)
    assert g["val"].tobytes() == ref.val.tobytes()
    if ref.row_scale is not None:
        assert g["row_scale"].tobytes() == ref.row_scale.tobytes()
    rec, kb = O.records(ref, 128)
    assert P.nrec == len(rec)
    assert np.array_equal(g["kblk_ptr"], kb)
    assert np.array_equal(g["rec"], rec)


def err(C_hat, C_ref, scale) -> float:
    return O.err_metric(np.asarray(C_hat, np.float64), C_ref, scale)


def threads() -> int:
    """Host threads for the full-size oracle runs (the GPU machine's CPU share)."""
    return max(1, min(16, O.max_threads()))


@functools.lru_cache(maxsize=None)
def cnn_reference(s: float):
    """(problem, C, |A||B|) of the 256 x 2304 x 3136 layer at sparsity s, full
    size, from the threaded FP64 oracle (cached across tests)."""
    from paper_2307_03930_amd import synth
    pr = synth.cnn_layer(s)
    t = threads()
    return pr, O.spmm(pr.A, pr.B, threads=t), O.abs_product(pr.A, pr.B, threads=t)


@functools.lru_cache(maxsize=None)
def precision_reference(s: float):
    """(problem, C on the FP32 source values, |A||B|) of the 4096 x 4096 x 2048
    precision form at sparsity s, full size."""
    from paper_2307_03930_amd import synth
    pr = synth.precision_problem(s)
    t = threads()
    return pr, O.spmm(pr.A, pr.B, threads=t), O.abs_product(pr.A, pr.B, threads=t)


def assert_nonfinite_match(C_hat: np.ndarray, C_ref: np.ndarray) -> np.ndarray:
    """The positions where the oracle is +Inf, -Inf or NaN must hold the same
    class on the GPU; returns the mask of positions finite in both."""
    C_hat = np.asarray(C_hat, np.float64)
    for f in (np.isnan, np.isposinf, np.isneginf):
        assert np.array_equal(f(C_hat), f(C_ref)), f.__name__
    return np.isfinite(C_ref)
