"""ctypes front end of the plain-C FP64 oracle (rosko_oracle.c).

TEST INFRASTRUCTURE ONLY (tests, the smoke check, the benchmark's CPU
baseline).  It shares no code with the HIP path.  `build()` compiles the C
file with gcc; `lib()` loads the result, building it first if absent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rosko_oracle.c")
SO = os.path.join(HERE, "librosko_oracle.so")

F32, BF16, FP8 = 0, 1, 2
_VAL_NP = {F32: np.float32, BF16: np.uint16, FP8: np.uint8}

_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(SO):
        tmp = SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(SO)
        p = C.c_void_p
        i64, i32 = C.c_int64, C.c_int32
        L.ro_is_nonzero.argtypes = [C.c_float]; L.ro_is_nonzero.restype = C.c_int
        L.ro_bf16_encode.argtypes = [C.c_float]; L.ro_bf16_encode.restype = C.c_uint16
        L.ro_bf16_decode.argtypes = [C.c_uint16]; L.ro_bf16_decode.restype = C.c_float
        L.ro_fp8_encode.argtypes = [C.c_float]; L.ro_fp8_encode.restype = C.c_uint8
        L.ro_fp8_decode.argtypes = [C.c_uint8]; L.ro_fp8_decode.restype = C.c_float
        L.ro_fp8_decode_d.argtypes = [C.c_uint8]; L.ro_fp8_decode_d.restype = C.c_double
        L.ro_row_scale.argtypes = [p, i64, i64, i64, p]; L.ro_row_scale.restype = None
        L.ro_pack_count.argtypes = [p, i64, i64, i64, i32, p]; L.ro_pack_count.restype = i64
        L.ro_pack.argtypes = [p, i64, i64, i64, i32, i32, p, p, p, p, p, p, p, p]
        L.ro_pack.restype = None
        L.ro_unpack.argtypes = [i64, i64, i32, i32, p, p, p, p, p, p, p, p]
        L.ro_unpack.restype = None
        L.ro_spmm_csr.argtypes = [p, i64, i64, i64, p, i64, i64, p]; L.ro_spmm_csr.restype = None
        L.ro_spmm_csr_par.argtypes = [p, i64, i64, i64, p, i64, i64, p, i32]
        L.ro_spmm_csr_par.restype = None
        L.ro_dense_mm.argtypes = [p, i64, i64, i64, p, i64, i64, p]; L.ro_dense_mm.restype = None
        L.ro_abs_product.argtypes = [p, i64, i64, i64, p, i64, i64, p]
        L.ro_abs_product.restype = None
        L.ro_spmm_packed.argtypes = [i64, i64, i32, i32, p, p, p, p, p, p, p, p, i64, i64, p,
                                     C.c_int, p]
        L.ro_spmm_packed.restype = None
        L.ro_grad_dB.argtypes = [p, i64, i64, i64, p, i64, i64, p]; L.ro_grad_dB.restype = None
        L.ro_grad_dA_packed.argtypes = [i64, i32, p, p, p, p, p, p, i64, p, i64, i64, p]
        L.ro_grad_dA_packed.restype = None
        L.ro_max_threads.argtypes = []; L.ro_max_threads.restype = i32
        L.ro_abs_product_par.argtypes = [p, i64, i64, i64, p, i64, i64, p, i32]
        L.ro_abs_product_par.restype = None
        L.ro_grad_dB_par.argtypes = [p, i64, i64, i64, p, i64, i64, p, i32]
        L.ro_grad_dB_par.restype = None
        L.ro_grad_dA_packed_par.argtypes = [i64, i32, p, p, p, p, p, p, i64, p, i64, i64, p,
                                            i32]
        L.ro_grad_dA_packed_par.restype = None
        L.ro_conv3x3.argtypes = [p, i64, i64, i64, i64, p, p, i32, i32]
        L.ro_conv3x3.restype = None
        L.ro_records.argtypes = [i64, i64, i32, i32, i32, p, p, p, p, p, p, p, p]
        L.ro_records.restype = i64
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------- encodings
def bf16_encode(x: float) -> int:
    return int(lib().ro_bf16_encode(C.c_float(x)))


def bf16_decode(h: int) -> float:
    return float(lib().ro_bf16_decode(C.c_uint16(h)))


def fp8_encode(y: float) -> int:
    return int(lib().ro_fp8_encode(C.c_float(y)))


def fp8_decode(c: int) -> float:
    return float(lib().ro_fp8_decode_d(C.c_uint8(c)))


def row_scale(A: np.ndarray) -> np.ndarray:
    A = _f32(A)
    M, K = A.shape
    out = np.empty(M, dtype=np.float32)
    lib().ro_row_scale(_ptr(A), M, K, K, _ptr(out))
    return out


# ------------------------------------------------------------------ packing
@dataclass
class Packed:
    """Oracle packed form of an M x K matrix (Alg. 1 per mr-row panel)."""
    M: int
    K: int
    mr: int
    dtype: int
    panel_nz_ptr: np.ndarray   # int64 [P+1]
    panel_col_ptr: np.ndarray  # int64 [P+1]
    col_ind: np.ndarray        # int32 [ncols]
    col_nnz: np.ndarray        # int32 [ncols]
    col_ptr: np.ndarray        # int64 [ncols+1]
    loc: np.ndarray            # uint8 [nnz]
    val: np.ndarray            # float32 / uint16 / uint8 [nnz]
    row_scale: np.ndarray | None  # float32 [M] (FP8 only)

    @property
    def nnz(self) -> int:
        return int(self.panel_nz_ptr[-1])

    @property
    def ncols(self) -> int:
        return int(self.panel_col_ptr[-1])

    @property
    def n_panels(self) -> int:
        return (self.M + self.mr - 1) // self.mr


def pack_count(A: np.ndarray, mr: int) -> tuple[int, int]:
    A = _f32(A)
    M, K = A.shape
    nc = C.c_int64(0)
    nnz = lib().ro_pack_count(_ptr(A), M, K, K, mr, C.byref(nc))
    return int(nnz), int(nc.value)


def pack(A: np.ndarray, mr: int, dtype: int = F32) -> Packed:
    A = _f32(A)
    M, K = A.shape
    nnz, ncols = pack_count(A, mr)
    P = (M + mr - 1) // mr
    pnz = np.zeros(P + 1, np.int64)
    pcol = np.zeros(P + 1, np.int64)
    ci = np.zeros(max(ncols, 1), np.int32)
    cn = np.zeros(max(ncols, 1), np.int32)
    cp = np.zeros(ncols + 1, np.int64)
    loc = np.zeros(max(nnz, 1), np.uint8)
    val = np.zeros(max(nnz, 1), _VAL_NP[dtype])
    rs = np.zeros(max(M, 1), np.float32) if dtype == FP8 else None
    lib().ro_pack(_ptr(A), M, K, K, mr, dtype, _ptr(pnz), _ptr(pcol), _ptr(ci), _ptr(cn),
                  _ptr(cp), _ptr(loc), _ptr(val), _ptr(rs))
    return Packed(M, K, mr, dtype, pnz, pcol, ci[:ncols], cn[:ncols], cp, loc[:nnz], val[:nnz],
                  None if rs is None else rs[:M])


KSTEP = 128   # K-block width of the derived record index


def records(pk: Packed, kstep: int = KSTEP):
    """(rec [nrec x 16] uint32, rec_kblk [P*(nkb+1)] int64): the column-record
    copy of the packed panels and its K-block index (see ro_records)."""
    L = lib()
    args = (pk.M, pk.K, pk.mr, pk.dtype, kstep, _ptr(pk.panel_col_ptr), _ptr(pk.col_ind),
            _ptr(pk.col_nnz), _ptr(pk.col_ptr), _ptr(pk.loc), _ptr(pk.val))
    nrec = L.ro_records(*args, None, None)
    nkb = (pk.K + kstep - 1) // kstep
    rec = np.zeros((max(nrec, 1), 16), np.uint32)
    kb = np.zeros(max(pk.n_panels * (nkb + 1), 1), np.int64)
    L.ro_records(*args, _ptr(rec), _ptr(kb))
    return rec[:nrec], kb[:pk.n_panels * (nkb + 1)]


def unpack(pk: Packed) -> np.ndarray:
    out = np.zeros((pk.M, pk.K), np.float64)
    lib().ro_unpack(pk.M, pk.K, pk.mr, pk.dtype, _ptr(pk.panel_col_ptr), _ptr(pk.col_ind),
                    _ptr(pk.col_nnz), _ptr(pk.col_ptr), _ptr(pk.loc), _ptr(pk.val),
                    _ptr(pk.row_scale), _ptr(out))
    return out


# --------------------------------------------------------------------- SpMM
def spmm(A: np.ndarray, B: np.ndarray, threads: int = 1) -> np.ndarray:
    """FP64 C = A*B over A's nonzeros (CSR, ascending k)."""
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    out = np.empty((M, N), np.float64)
    if threads > 1:
        lib().ro_spmm_csr_par(_ptr(A), M, K, K, _ptr(B), N, N, _ptr(out), threads)
    else:
        lib().ro_spmm_csr(_ptr(A), M, K, K, _ptr(B), N, N, _ptr(out))
    return out


def dense_mm(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    _, N = B.shape
    out = np.empty((M, N), np.float64)
    lib().ro_dense_mm(_ptr(A), M, K, K, _ptr(B), N, N, _ptr(out))
    return out


def abs_product(A: np.ndarray, B: np.ndarray, threads: int = 1) -> np.ndarray:
    A, B = _f32(A), _f32(B)
    M, K = A.shape
    _, N = B.shape
    out = np.empty((M, N), np.float64)
    if threads > 1:
        lib().ro_abs_product_par(_ptr(A), M, K, K, _ptr(B), N, N, _ptr(out), threads)
    else:
        lib().ro_abs_product(_ptr(A), M, K, K, _ptr(B), N, N, _ptr(out))
    return out


def spmm_packed(pk: Packed, B: np.ndarray, C_in: np.ndarray | None = None) -> np.ndarray:
    """Alg. 2 over the oracle's packed arrays; decoded values; FP64."""
    B = _f32(B)
    N = B.shape[1]
    out = np.empty((pk.M, N), np.float64)
    cin = None if C_in is None else np.ascontiguousarray(C_in, np.float64)
    lib().ro_spmm_packed(pk.M, pk.K, pk.mr, pk.dtype, _ptr(pk.panel_col_ptr), _ptr(pk.col_ind),
                         _ptr(pk.col_nnz), _ptr(pk.col_ptr), _ptr(pk.loc), _ptr(pk.val),
                         _ptr(pk.row_scale), _ptr(B), N, N, _ptr(cin), 0 if cin is None else 1,
                         _ptr(out))
    return out


# ----------------------------------------------------------------- backward
def grad_dB(A: np.ndarray, dC: np.ndarray, threads: int = 1) -> np.ndarray:
    A, dC = _f32(A), _f32(dC)
    M, K = A.shape
    N = dC.shape[1]
    out = np.empty((K, N), np.float64)
    if threads > 1:
        lib().ro_grad_dB_par(_ptr(A), M, K, K, _ptr(dC), N, N, _ptr(out), threads)
    else:
        lib().ro_grad_dB(_ptr(A), M, K, K, _ptr(dC), N, N, _ptr(out))
    return out


def grad_dA_packed(pk: Packed, dC: np.ndarray, B: np.ndarray, threads: int = 1) -> np.ndarray:
    dC, B = _f32(dC), _f32(B)
    N = B.shape[1]
    out = np.empty(max(pk.nnz, 1), np.float64)
    args = (pk.M, pk.mr, _ptr(pk.panel_col_ptr), _ptr(pk.col_ind), _ptr(pk.col_nnz),
            _ptr(pk.col_ptr), _ptr(pk.loc), _ptr(dC), N, _ptr(B), N, N, _ptr(out))
    if threads > 1:
        lib().ro_grad_dA_packed_par(*args, threads)
    else:
        lib().ro_grad_dA_packed(*args)
    return out[:pk.nnz]


def max_threads() -> int:
    return int(lib().ro_max_threads())


# ------------------------------------------------------------ error metric
def err_metric(C_hat: np.ndarray, C_ref: np.ndarray, scale: np.ndarray) -> float:
    """max_i |C_hat_i - C_ref_i| / scale_i, with 0/0 counted as 0; `scale` is
    (|A| |B|)_i, the natural scale of a componentwise rounding bound."""
    d = np.abs(np.asarray(C_hat, np.float64) - C_ref)
    s = np.asarray(scale, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(s > 0, d / np.where(s > 0, s, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


# ------------------------------------------------------------ CSR input
def _csr_rows(row_ptr, col_idx, val, B, rows, absolute: bool) -> np.ndarray:
    B = _f32(B).astype(np.float64)
    if absolute:
        B = np.abs(B)
    out = np.zeros((len(rows), B.shape[1]), np.float64)
    for i, m in enumerate(rows):
        b, e = int(row_ptr[m]), int(row_ptr[m + 1])
        a = np.asarray(val[b:e], np.float32).astype(np.float64)
        if absolute:
            a = np.abs(a)
        out[i] = a @ B[np.asarray(col_idx[b:e], np.int64)]
    return out


def spmm_csr_rows(row_ptr, col_idx, val, B, rows) -> np.ndarray:
    """Rows `rows` of C = A B in FP64 for A given in CSR form, by the
    definition of the product (Sec. 3): C[m] is the sum over the stored
    entries (m, k, a) of row m of a * B[k]."""
    return _csr_rows(row_ptr, col_idx, val, B, rows, False)


def abs_spmm_csr_rows(row_ptr, col_idx, val, B, rows) -> np.ndarray:
    """The same rows of |A| |B| (the error scale of a computed product)."""
    return _csr_rows(row_ptr, col_idx, val, B, rows, True)


# ----------------------------------------------------- direct convolution
def conv3x3_direct(A: np.ndarray, X: np.ndarray, threads: int = 1,
                   absolute: bool = False) -> np.ndarray:
    """FP64 direct 3x3 convolution (stride 1, zero padding 1) of X (C_in, H,
    W) with the weight matrix A (C_out x C_in*9, column c*9 + ky*3 + kx) over
    A's kept entries: the product the method computes without im2col (Sec. 1).
    absolute: the same sum of |weight| |input| (the error scale).
    Returns (C_out, H, W)."""
    A, X = _f32(A), _f32(X)
    C_out, K = A.shape
    C_in, H, W = X.shape
    assert K == 9 * C_in
    out = np.empty((C_out, H, W), np.float64)
    lib().ro_conv3x3(_ptr(A), C_out, C_in, H, W, _ptr(X), _ptr(out), 1 if absolute else 0,
                     max(1, threads))
    return out
