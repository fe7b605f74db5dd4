"""Torch-facing wrappers of the C ABI: device memory and streams come from
torch, every step of the computation runs in librosko.so.

  pack(A, mr, dtype)            Alg. 1 on the GPU -> PackedMatrix
  pack_transpose(A, mr)         packs A^T (for dB = A^T dC)
  spmm(P, B, C=None, beta=0)    Alg. 2 on the GPU: C = A B (or C += A B)
  spmm_backward(P, Pt, B, dC)   dB = A^T dC and dA (packed order)
  pack_csr(row_ptr, col, val)   Alg. 1 from CSR input (graphs), optional row order
  row_order(row_ptr, mr, mode)  the inspector's row order for pack_csr
  ConvLayer(P, C_in, H, W)      sparse direct 3x3 convolution (no im2col)
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

DTYPES = {"f32": L.ROSKO_F32, "bf16": L.ROSKO_BF16, "fp8": L.ROSKO_FP8_E4M3}
_VAL_TORCH = {L.ROSKO_F32: torch.float32, L.ROSKO_BF16: torch.int16,
              L.ROSKO_FP8_E4M3: torch.uint8}


def _stream_ptr(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dtype_code(dtype) -> int:
    if isinstance(dtype, str):
        return DTYPES[dtype]
    return int(dtype)


@dataclass
class PackedMatrix:
    """A packed M x K matrix: the device arrays of include/rosko.h's
    rosko_packed, owned here as torch tensors."""
    M: int
    K: int
    mr: int
    val_dtype: int
    nnz: int
    ncols: int
    nrec: int
    panel_nz_ptr: torch.Tensor
    panel_col_ptr: torch.Tensor
    col_ind: torch.Tensor
    col_nnz: torch.Tensor
    col_ptr: torch.Tensor
    loc: torch.Tensor
    val: torch.Tensor
    row_scale: torch.Tensor | None
    kblk_ptr: torch.Tensor
    rec: torch.Tensor
    row_perm: torch.Tensor | None = None   # packed row i holds matrix row row_perm[i]

    @property
    def n_panels(self) -> int:
        return (self.M + self.mr - 1) // self.mr

    def struct(self) -> L.RoskoPacked:
        s = L.RoskoPacked()
        s.M, s.K, s.mr, s.n_panels = self.M, self.K, self.mr, self.n_panels
        s.val_dtype = self.val_dtype
        s.nnz_cap, s.ncols_cap, s.nrec_cap = self.nnz, self.ncols, self.nrec
        s.nnz, s.ncols, s.nrec = self.nnz, self.ncols, self.nrec
        s.panel_nz_ptr = self.panel_nz_ptr.data_ptr()
        s.panel_col_ptr = self.panel_col_ptr.data_ptr()
        s.col_ind = self.col_ind.data_ptr()
        s.col_nnz = self.col_nnz.data_ptr()
        s.col_ptr = self.col_ptr.data_ptr()
        s.loc = self.loc.data_ptr()
        s.val = self.val.data_ptr()
        s.row_scale = 0 if self.row_scale is None else self.row_scale.data_ptr()
        s.kblk_ptr = self.kblk_ptr.data_ptr()
        s.rec = self.rec.data_ptr()
        s.row_perm = 0 if self.row_perm is None else self.row_perm.data_ptr()
        return s

    def values(self) -> torch.Tensor:
        """The nnz stored values (raw encoding)."""
        return self.val[: self.nnz]


def workspace_size(M: int, K: int, mr: int, transpose: bool = False) -> int:
    n = C.c_size_t(0)
    L.check(L.lib().rosko_pack_workspace_size(M, K, mr, 1 if transpose else 0, C.byref(n)))
    return int(n.value)


def _check_dense(A: torch.Tensor, name: str):
    if not (A.is_cuda and A.dtype == torch.float32 and A.dim() == 2):
        raise ValueError(f"{name} must be a 2-D float32 CUDA tensor")
    if A.stride(1) != 1:
        raise ValueError(f"{name} must be row-major with unit column stride")


def _alloc(M, K, mr, dtype, nnz, ncols, nrec, device):
    P = (M + mr - 1) // mr
    nkb = (K + L.ROSKO_KSTEP - 1) // L.ROSKO_KSTEP
    i64, i32 = torch.int64, torch.int32
    return PackedMatrix(
        M=M, K=K, mr=mr, val_dtype=dtype, nnz=nnz, ncols=ncols, nrec=nrec,
        panel_nz_ptr=torch.empty(P + 1, dtype=i64, device=device),
        panel_col_ptr=torch.empty(P + 1, dtype=i64, device=device),
        col_ind=torch.empty(max(ncols, 1), dtype=i32, device=device),
        col_nnz=torch.empty(max(ncols, 1), dtype=i32, device=device),
        col_ptr=torch.empty(ncols + 1, dtype=i64, device=device),
        loc=torch.zeros(max(nnz, 1), dtype=torch.uint8, device=device),
        val=torch.zeros(max(nnz, 1), dtype=_VAL_TORCH[dtype], device=device),
        row_scale=(torch.empty(max(M, 1), dtype=torch.float32, device=device)
                   if dtype == L.ROSKO_FP8_E4M3 else None),
        kblk_ptr=torch.empty(max(P * (nkb + 1), 1), dtype=i64, device=device),
        rec=torch.empty((max(nrec, 1), 16), dtype=torch.int32, device=device),
    )


def pack_query(A: torch.Tensor, mr: int, ws: torch.Tensor | None = None):
    """(nnz, ncols, nrec) of packing A with panel height mr.  Synchronises."""
    _check_dense(A, "A")
    M, K = A.shape
    if ws is None:
        ws = torch.empty(max(workspace_size(M, K, mr), 1), dtype=torch.uint8, device=A.device)
    nnz, ncols, nrec = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    L.check(L.lib().rosko_pack_query(_ptr(A), M, K, max(A.stride(0), 1), mr, _ptr(ws), ws.numel(),
                                     _stream_ptr(), C.byref(nnz), C.byref(ncols), C.byref(nrec)))
    return int(nnz.value), int(ncols.value), int(nrec.value)


def pack(A: torch.Tensor, mr: int = 32, dtype="f32") -> PackedMatrix:
    """Alg. 1 on every mr-row panel of A (2-D float32 CUDA tensor)."""
    _check_dense(A, "A")
    dt = _dtype_code(dtype)
    M, K = A.shape
    ws = torch.empty(max(workspace_size(M, K, mr), 1), dtype=torch.uint8, device=A.device)
    nnz, ncols, nrec = pack_query(A, mr, ws)
    P = _alloc(M, K, mr, dt, nnz, ncols, nrec, A.device)
    st = P.struct()
    L.check(L.lib().rosko_pack(_ptr(A), M, K, max(A.stride(0), 1), mr, dt, _ptr(ws), ws.numel(),
                               C.byref(st), _stream_ptr()))
    P._ws = ws  # keep the workspace alive until the enqueued work is done
    return P


def pack_transpose(A: torch.Tensor, mr: int = 32) -> PackedMatrix:
    """Packs A^T (K x M, FP32 values) directly from A."""
    _check_dense(A, "A")
    M, K = A.shape
    ws = torch.empty(max(workspace_size(M, K, mr, transpose=True), 1), dtype=torch.uint8,
                     device=A.device)
    nnz, ncols, nrec = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    L.check(L.lib().rosko_pack_transpose_query(_ptr(A), M, K, max(A.stride(0), 1), mr,
                                               _ptr(ws), ws.numel(), _stream_ptr(),
                                               C.byref(nnz), C.byref(ncols), C.byref(nrec)))
    nnz, ncols, nrec = int(nnz.value), int(ncols.value), int(nrec.value)
    P = _alloc(K, M, mr, L.ROSKO_F32, nnz, ncols, nrec, A.device)
    st = P.struct()
    L.check(L.lib().rosko_pack_transpose(_ptr(A), M, K, max(A.stride(0), 1), mr, L.ROSKO_F32, _ptr(ws),
                                         ws.numel(), C.byref(st), _stream_ptr()))
    P._ws = ws
    return P


def make_plan(cols_per_lane: int | None = None, waves_per_tile: int | None = None,
              k_split: int | None = None, depth: int | None = None,
              path: int = L.ROSKO_PATH_SPARSE):
    """A rosko_plan; None (automatic) when nothing is given.  A field left
    None is the library's choice (0), columns per lane defaulting to 4."""
    if cols_per_lane is None and waves_per_tile is None and k_split is None and depth is None:
        return None
    p = L.RoskoPlan()
    p.path = path
    p.cols_per_lane = cols_per_lane or 4
    p.waves_per_tile = waves_per_tile or 0
    p.k_split = k_split or 0
    p.depth = depth or 0
    return p


def dense_plan():
    """The plan of the dense-MFMA path (every panel densified, matrix cores)."""
    p = L.RoskoPlan()
    p.path = L.ROSKO_PATH_DENSE
    p.cols_per_lane, p.waves_per_tile, p.k_split, p.depth = 0, 0, 1, 0
    return p


def spmm_workspace_size(P: PackedMatrix, N: int, plan=None) -> int:
    n = C.c_size_t(0)
    st = P.struct()
    L.check(L.lib().rosko_spmm_workspace_size(C.byref(st), N,
                                              C.byref(plan) if plan is not None else None,
                                              C.byref(n)))
    return int(n.value)


def spmm(P: PackedMatrix, B: torch.Tensor, C_out: torch.Tensor | None = None, beta: int = 0,
         plan=None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """C = A B (beta 0) or C += A B (beta 1).  B: K x N float32 or bfloat16."""
    if not (B.is_cuda and B.dim() == 2 and (B.stride(1) == 1 or B.numel() == 0)):
        raise ValueError("B must be a 2-D row-major CUDA tensor")
    if B.dtype == torch.float32:
        bdt = L.ROSKO_F32
    elif B.dtype == torch.bfloat16:
        bdt = L.ROSKO_BF16
    else:
        raise ValueError("B must be float32 or bfloat16")
    if B.shape[0] != P.K:
        raise ValueError(f"B has {B.shape[0]} rows, A has {P.K} columns")
    N = B.shape[1]
    if C_out is None:
        if beta:
            raise ValueError("beta = 1 needs C_out")
        C_out = torch.empty((P.M, N), dtype=torch.float32, device=B.device)
    need = spmm_workspace_size(P, N, plan)
    if need and (ws is None or ws.numel() < need):
        ws = torch.empty(need, dtype=torch.uint8, device=B.device)
    st = P.struct()
    pl = C.byref(plan) if plan is not None else None
    L.check(L.lib().rosko_spmm(C.byref(st), _ptr(B), bdt, N, max(B.stride(0), 1), _ptr(C_out),
                               max(C_out.stride(0), 1), beta, pl,
                               _ptr(ws) if need else None, ws.numel() if need else 0,
                               _stream_ptr()))
    return C_out


def spmm_backward(P: PackedMatrix, Pt: PackedMatrix | None, B: torch.Tensor, dC: torch.Tensor,
                  need_dB: bool = True, need_dA: bool = True, ws: torch.Tensor | None = None):
    """(dA in packed order, dB) for C = A B."""
    N = dC.shape[1]
    dB = torch.empty((P.K, N), dtype=torch.float32, device=dC.device) if need_dB else None
    dA = torch.empty(max(P.nnz, 1), dtype=torch.float32, device=dC.device) if need_dA else None
    st = P.struct()
    stt = Pt.struct() if (Pt is not None and need_dB) else None
    n = C.c_size_t(0)
    L.check(L.lib().rosko_spmm_backward_workspace_size(
        C.byref(st) if need_dA else None, C.byref(stt) if stt is not None else None, N,
        C.byref(n)))
    need = int(n.value)
    if need and (ws is None or ws.numel() < need):
        ws = torch.empty(need, dtype=torch.uint8, device=dC.device)
    L.check(L.lib().rosko_spmm_backward(
        C.byref(st), C.byref(stt) if stt is not None else None, _ptr(B),
        max(B.stride(0), 1), _ptr(dC), max(dC.stride(0), 1), N, _ptr(dB),
        max(dB.stride(0), 1) if dB is not None else 1, _ptr(dA),
        dA.numel() if dA is not None else 0,
        _ptr(ws) if need else None, ws.numel() if need else 0, _stream_ptr()))
    return (dA[: P.nnz] if dA is not None else None), dB


PACK_MODES = {"auto": L.ROSKO_PACK_AUTO, "two_pass": L.ROSKO_PACK_TWO_PASS,
              "recount": L.ROSKO_PACK_RECOUNT}


def set_pack_mode(mode: str) -> None:
    """Process-wide: how packing enqueues its running offsets (rosko_pack_set_mode):
    "auto" (one launch where the grid allows), "two_pass" (count, then write)
    or "recount" (one launch, every tile counting the tiles before it; for
    tests).  The packed arrays are the same in every mode."""
    L.check(L.lib().rosko_pack_set_mode(PACK_MODES[mode]))


def pack_into(A: torch.Tensor, P: PackedMatrix, ws: torch.Tensor) -> PackedMatrix:
    """Re-packs A into P's existing buffers (same shape, mr and dtype; the
    capacities must hold A's structure).  Asynchronous: no host sync."""
    _check_dense(A, "A")
    M, K = A.shape
    if (M, K) != (P.M, P.K):
        raise ValueError("shape differs from the packed buffers")
    st = P.struct()
    L.check(L.lib().rosko_pack(_ptr(A), M, K, max(A.stride(0), 1), P.mr, P.val_dtype, _ptr(ws),
                               ws.numel(), C.byref(st), _stream_ptr()))
    return P


def pack_batch_into(items) -> None:
    """Re-packs several matrices at once (rosko_pack_batch): items is a
    sequence of (A, P, ws) as for pack_into, or (A, Pt, ws, True) as for
    pack_transpose_into (FP32 values), with distinct workspaces and buffers.
    The packed arrays are those the one-matrix calls give, bit for bit; the
    single passes of matrices of one kernel form share launches.
    Asynchronous: no host sync."""
    items = list(items)
    if len(items) > L.ROSKO_PACK_BATCH_MAX:
        raise ValueError(f"at most {L.ROSKO_PACK_BATCH_MAX} matrices per batch")
    jobs = (L.RoskoPackJob * max(len(items), 1))()
    structs = []
    for i, item in enumerate(items):
        A, P, ws = item[:3]
        tr = bool(item[3]) if len(item) > 3 else False
        _check_dense(A, "A")
        M, K = A.shape
        if ((K, M) if tr else (M, K)) != (P.M, P.K):
            raise ValueError("shape differs from the packed buffers")
        if tr and P.val_dtype != L.ROSKO_F32:
            raise ValueError("transposed packs hold FP32 values")
        st = P.struct()
        structs.append(st)
        jobs[i] = L.RoskoPackJob(_ptr(A), M, K, max(A.stride(0), 1), P.mr, P.val_dtype,
                                 1 if tr else 0, 0, _ptr(ws), ws.numel(), C.pointer(st))
    L.check(L.lib().rosko_pack_batch(len(items), jobs, _stream_ptr()))


def pack_transpose_into(A: torch.Tensor, Pt: PackedMatrix, ws: torch.Tensor) -> PackedMatrix:
    """Re-packs A^T (A: M x K) into Pt's existing buffers (Pt is K x M, FP32
    values; its capacities must hold A's structure).  Asynchronous."""
    _check_dense(A, "A")
    M, K = A.shape
    if (K, M) != (Pt.M, Pt.K):
        raise ValueError("shape differs from the packed transpose buffers")
    st = Pt.struct()
    L.check(L.lib().rosko_pack_transpose(_ptr(A), M, K, max(A.stride(0), 1), Pt.mr,
                                         L.ROSKO_F32, _ptr(ws), ws.numel(), C.byref(st),
                                         _stream_ptr()))
    return Pt


def pack_result(P: PackedMatrix, ws: torch.Tensor, transpose: bool = False) -> tuple[int, int]:
    """Synchronises; (nnz, ncols) of the last pack_into (pack_transpose_into
    with transpose=True) with this workspace.  Raises if they exceeded P's
    capacities."""
    st = P.struct()
    L.check(L.lib().rosko_pack_result(_ptr(ws), ws.numel(), C.byref(st), _stream_ptr()))
    return int(st.nnz), int(st.ncols)


def scatter_dense(P: PackedMatrix, vals: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """out[m][k] = vals[z] for every stored entry z of P (packed order); the
    other entries of out are left as they are."""
    if not (out.is_cuda and out.dtype == torch.float32 and out.dim() == 2
            and out.shape == (P.M, P.K) and (out.stride(1) == 1 or out.numel() == 0)):
        raise ValueError("out must be a row-major float32 CUDA tensor of A's shape")
    if vals.dtype != torch.float32 or not vals.is_cuda:
        raise ValueError("vals must be a float32 CUDA tensor")
    st = P.struct()
    L.check(L.lib().rosko_scatter_dense(C.byref(st), _ptr(vals), vals.numel(), _ptr(out),
                                        max(out.stride(0), 1), _stream_ptr()))
    return out


# ------------------------------------------------------------ CSR input

ORDERS = {"degree": L.ROSKO_ORDER_DEGREE, "balanced": L.ROSKO_ORDER_BALANCED}


def _check_csr(row_ptr, col_idx, val):
    ok = (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.dim() == 1
          and row_ptr.is_contiguous() and col_idx.is_cuda and col_idx.dtype == torch.int32
          and col_idx.is_contiguous() and val.is_cuda and val.dtype == torch.float32
          and val.is_contiguous() and col_idx.numel() == val.numel())
    if not ok:
        raise ValueError("CSR input: row_ptr int64, col_idx int32 and val float32 contiguous "
                         "CUDA tensors, col_idx and val of one length")


def csr_workspace_size(M: int, K: int, nnz_in: int, mr: int) -> int:
    n = C.c_size_t(0)
    L.check(L.lib().rosko_pack_csr_workspace_size(M, K, nnz_in, mr, C.byref(n)))
    return int(n.value)


def pack_csr(row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor, K: int,
             mr: int = 8, dtype="f32", perm: torch.Tensor | None = None) -> PackedMatrix:
    """Alg. 1 on the CSR matrix (M = len(row_ptr) - 1 rows, K columns), its
    packed row i taken from CSR row perm[i] when perm is given; the result's
    SpMM writes C in the matrix's own row order.  Synchronises (sizing)."""
    _check_csr(row_ptr, col_idx, val)
    if perm is not None and not (perm.is_cuda and perm.dtype == torch.int32
                                 and perm.is_contiguous()):
        raise ValueError("perm must be a contiguous int32 CUDA tensor")
    dt = _dtype_code(dtype)
    M = row_ptr.numel() - 1
    nz = col_idx.numel()
    ws = torch.empty(max(csr_workspace_size(M, K, nz, mr), 1), dtype=torch.uint8,
                     device=row_ptr.device)
    nnz, ncols, nrec = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    L.check(L.lib().rosko_pack_csr_query(
        _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(perm), M, K, nz, mr, _ptr(ws), ws.numel(),
        _stream_ptr(), C.byref(nnz), C.byref(ncols), C.byref(nrec)))
    P = _alloc(M, K, mr, dt, int(nnz.value), int(ncols.value), int(nrec.value),
               row_ptr.device)
    P.row_perm = perm
    st = P.struct()
    L.check(L.lib().rosko_pack_csr(_ptr(row_ptr), _ptr(col_idx), _ptr(val), M, K, nz, mr, dt,
                                   _ptr(ws), ws.numel(), C.byref(st), _stream_ptr()))
    L.check(L.lib().rosko_pack_csr_result(_ptr(ws), ws.numel(), C.byref(st), _stream_ptr()))
    P.nnz, P.ncols, P.nrec = int(st.nnz), int(st.ncols), int(st.nrec)
    P._ws = ws
    return P


def pack_csr_into(row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor,
                  P: PackedMatrix, ws: torch.Tensor) -> PackedMatrix:
    """Re-packs a CSR matrix of the same shape into P's buffers (P.row_perm
    as the row order).  Asynchronous."""
    _check_csr(row_ptr, col_idx, val)
    st = P.struct()
    L.check(L.lib().rosko_pack_csr(_ptr(row_ptr), _ptr(col_idx), _ptr(val), P.M, P.K,
                                   col_idx.numel(), P.mr, P.val_dtype, _ptr(ws), ws.numel(),
                                   C.byref(st), _stream_ptr()))
    return P


def row_order(row_ptr: torch.Tensor, mr: int, mode: str = "balanced") -> torch.Tensor:
    """The inspector's row order (int32 permutation) for pack_csr."""
    if not (row_ptr.is_cuda and row_ptr.dtype == torch.int64 and row_ptr.is_contiguous()):
        raise ValueError("row_ptr must be a contiguous int64 CUDA tensor")
    M = row_ptr.numel() - 1
    n = C.c_size_t(0)
    L.check(L.lib().rosko_row_order_workspace_size(M, C.byref(n)))
    ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=row_ptr.device)
    perm = torch.empty(max(M, 1), dtype=torch.int32, device=row_ptr.device)
    L.check(L.lib().rosko_row_order(_ptr(row_ptr), M, mr, ORDERS[mode], _ptr(ws), ws.numel(),
                                    _ptr(perm), _stream_ptr()))
    return perm[:M]


# ------------------------------------------------- direct convolution

def conv_geometry(C_in: int, H: int, W: int) -> tuple[int, int]:
    """(Wq, T): the padded row pitch and the length of each input copy."""
    wq, t = C.c_int64(0), C.c_int64(0)
    L.check(L.lib().rosko_conv_geometry(C_in, H, W, C.byref(wq), C.byref(t)))
    return int(wq.value), int(t.value)


class ConvLayer:
    """A pruned 3x3 convolution (stride 1, padding 1) run as the sparse
    direct convolution: P is the packed weight matrix (C_out x 9 C_in, the
    im2col column order), whose records are remapped once for the input size
    (C_in, H, W); run(X) returns the output on the padded-pitch grid
    (C_out x H*Wq), unpad() the C_out x H x W output."""

    def __init__(self, P: PackedMatrix, C_in: int, H: int, W: int, plan=None):
        self.P, self.C_in, self.H, self.W, self.plan = P, C_in, H, W, plan
        self.Wq, self.T = conv_geometry(C_in, H, W)
        dev = P.rec.device
        self.rec = torch.empty((max(P.nrec, 1), 16), dtype=torch.int32, device=dev)
        self.Bc = torch.empty(4 * self.T, dtype=torch.float32, device=dev)
        n = C.c_size_t(0)
        st = P.struct()
        L.check(L.lib().rosko_conv_workspace_size(C.byref(st), H, W,
                                                  C.byref(plan) if plan is not None else None,
                                                  C.byref(n)))
        self.ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=dev)
        self.ws_bytes = int(n.value)
        self.remap()

    def remap(self):
        """Rewrites the records for the input geometry (after a repack of P)."""
        st = self.P.struct()
        L.check(L.lib().rosko_conv_records(C.byref(st), self.C_in, self.H, self.W,
                                           _ptr(self.rec), self.rec.shape[0], _stream_ptr()))

    def run(self, X: torch.Tensor, out: torch.Tensor | None = None, beta: int = 0):
        if not (X.is_cuda and X.dtype == torch.float32 and X.is_contiguous()
                and tuple(X.shape) == (self.C_in, self.H, self.W)):
            raise ValueError("X must be a contiguous float32 CUDA tensor of (C_in, H, W)")
        L.check(L.lib().rosko_conv_input(_ptr(X), self.C_in, self.H, self.W, _ptr(self.Bc),
                                         _stream_ptr()))
        N = self.H * self.Wq
        if out is None:
            if beta:
                raise ValueError("beta = 1 needs out")
            out = torch.empty((self.P.M, N), dtype=torch.float32, device=X.device)
        st = self.P.struct()
        pl = C.byref(self.plan) if self.plan is not None else None
        L.check(L.lib().rosko_conv(C.byref(st), _ptr(self.rec), _ptr(self.Bc), self.C_in,
                                   self.H, self.W, _ptr(out), max(out.stride(0), 1), beta, pl,
                                   _ptr(self.ws) if self.ws_bytes else None, self.ws_bytes,
                                   _stream_ptr()))
        return out

    def unpad(self, Yq: torch.Tensor) -> torch.Tensor:
        Y = torch.empty((self.P.M, self.H, self.W), dtype=torch.float32, device=Yq.device)
        L.check(L.lib().rosko_conv_unpad(_ptr(Yq), max(Yq.stride(0), 1), self.P.M, self.H,
                                         self.W, _ptr(Y), _stream_ptr()))
        return Y
