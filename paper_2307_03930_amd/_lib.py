"""ctypes loader for librosko.so and the C structs of include/rosko.h.

Argument marshalling only.  There is no fallback: if the library is missing
the import of the ops fails with an error naming the build step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librosko.so")

ROSKO_OK = 0
ROSKO_EINVAL = -1
ROSKO_EUNSUPPORTED = -2
ROSKO_ESMALLBUF = -3
ROSKO_EHIP = -4
ROSKO_EINTERNAL = -5

ROSKO_F32 = 0
ROSKO_BF16 = 1
ROSKO_FP8_E4M3 = 2

ROSKO_PATH_AUTO = -1
ROSKO_PATH_SPARSE = 0
ROSKO_PATH_DENSE = 1
ROSKO_ORDER_DEGREE = 0
ROSKO_ORDER_BALANCED = 1
ROSKO_PACK_AUTO = 0
ROSKO_PACK_TWO_PASS = 1
ROSKO_PACK_RECOUNT = 2
ROSKO_PACK_BATCH_MAX = 64
ROSKO_NFEAT = 16
ROSKO_SCHED_CANDIDATES = 7
ROSKO_KSTEP = 128


class RoskoPacked(C.Structure):
    _fields_ = [
        ("M", C.c_int64), ("K", C.c_int64),
        ("mr", C.c_int32), ("n_panels", C.c_int32),
        ("val_dtype", C.c_int32), ("reserved", C.c_int32),
        ("nnz_cap", C.c_int64), ("ncols_cap", C.c_int64), ("nrec_cap", C.c_int64),
        ("nnz", C.c_int64), ("ncols", C.c_int64), ("nrec", C.c_int64),
        ("panel_nz_ptr", C.c_void_p), ("panel_col_ptr", C.c_void_p),
        ("col_ind", C.c_void_p), ("col_nnz", C.c_void_p), ("col_ptr", C.c_void_p),
        ("loc", C.c_void_p), ("val", C.c_void_p), ("row_scale", C.c_void_p),
        ("kblk_ptr", C.c_void_p), ("rec", C.c_void_p), ("row_perm", C.c_void_p),
    ]


class RoskoPackJob(C.Structure):
    _fields_ = [("A", C.c_void_p), ("M", C.c_int64), ("K", C.c_int64), ("lda", C.c_int64),
                ("mr", C.c_int32), ("val_dtype", C.c_int32), ("transpose", C.c_int32),
                ("reserved", C.c_int32), ("ws", C.c_void_p),
                ("ws_bytes", C.c_size_t), ("out", C.POINTER(RoskoPacked))]


class RoskoPlan(C.Structure):
    _fields_ = [("path", C.c_int32), ("cols_per_lane", C.c_int32),
                ("waves_per_tile", C.c_int32), ("k_split", C.c_int32),
                ("depth", C.c_int32)]


class RoskoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


_STATUS = {0: "ROSKO_OK", -1: "ROSKO_EINVAL", -2: "ROSKO_EUNSUPPORTED", -3: "ROSKO_ESMALLBUF",
           -4: "ROSKO_EHIP", -5: "ROSKO_EINTERNAL"}


def status_name(s: int) -> str:
    return _STATUS.get(s, f"status {s}")


_lib = None

# (name, restype, argtypes) for every entry point of include/rosko.h
_P, _I64, _I32, _SZ = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
SIGNATURES = {
    "rosko_pack_workspace_size": (_I32, [_I64, _I64, _I32, _I32, C.POINTER(_SZ)]),
    "rosko_pack_query": (_I32, [_P, _I64, _I64, _I64, _I32, _P, _SZ, _P,
                                C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "rosko_pack_transpose_query": (_I32, [_P, _I64, _I64, _I64, _I32, _P, _SZ, _P,
                                          C.POINTER(_I64), C.POINTER(_I64),
                                          C.POINTER(_I64)]),
    "rosko_pack": (_I32, [_P, _I64, _I64, _I64, _I32, _I32, _P, _SZ, C.POINTER(RoskoPacked), _P]),
    "rosko_pack_transpose": (_I32, [_P, _I64, _I64, _I64, _I32, _I32, _P, _SZ,
                                    C.POINTER(RoskoPacked), _P]),
    "rosko_pack_result": (_I32, [_P, _SZ, C.POINTER(RoskoPacked), _P]),
    "rosko_pack_set_mode": (_I32, [_I32]),
    "rosko_pack_batch": (_I32, [_I32, C.POINTER(RoskoPackJob), _P]),
    "rosko_pack_csr_workspace_size": (_I32, [_I64, _I64, _I64, _I32, C.POINTER(_SZ)]),
    "rosko_pack_csr_query": (_I32, [_P, _P, _P, _P, _I64, _I64, _I64, _I32, _P, _SZ, _P,
                                    C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "rosko_pack_csr": (_I32, [_P, _P, _P, _I64, _I64, _I64, _I32, _I32, _P, _SZ,
                              C.POINTER(RoskoPacked), _P]),
    "rosko_pack_csr_result": (_I32, [_P, _SZ, C.POINTER(RoskoPacked), _P]),
    "rosko_row_order_workspace_size": (_I32, [_I64, C.POINTER(_SZ)]),
    "rosko_row_order": (_I32, [_P, _I64, _I32, _I32, _P, _SZ, _P, _P]),
    "rosko_conv_geometry": (_I32, [_I32, _I32, _I32, C.POINTER(_I64), C.POINTER(_I64)]),
    "rosko_conv_input": (_I32, [_P, _I32, _I32, _I32, _P, _P]),
    "rosko_conv_records": (_I32, [C.POINTER(RoskoPacked), _I32, _I32, _I32, _P, _I64, _P]),
    "rosko_conv_workspace_size": (_I32, [C.POINTER(RoskoPacked), _I32, _I32,
                                         C.POINTER(RoskoPlan), C.POINTER(_SZ)]),
    "rosko_conv": (_I32, [C.POINTER(RoskoPacked), _P, _P, _I32, _I32, _I32, _P, _I64, _I32,
                          C.POINTER(RoskoPlan), _P, _SZ, _P]),
    "rosko_conv_unpad": (_I32, [_P, _I64, _I64, _I32, _I32, _P, _P]),
    "rosko_spmm_workspace_size": (_I32, [C.POINTER(RoskoPacked), _I64, C.POINTER(RoskoPlan),
                                         C.POINTER(_SZ)]),
    "rosko_spmm": (_I32, [C.POINTER(RoskoPacked), _P, _I32, _I64, _I64, _P, _I64, _I32,
                          C.POINTER(RoskoPlan), _P, _SZ, _P]),
    "rosko_spmm_noalloc": (_I32, [C.POINTER(RoskoPacked), _P, _I32, _I64, _I64, _P, _I64, _I32,
                                  C.POINTER(RoskoPlan), _P]),
    "rosko_spmm_backward_workspace_size": (_I32, [C.POINTER(RoskoPacked),
                                                  C.POINTER(RoskoPacked), _I64,
                                                  C.POINTER(_SZ)]),
    "rosko_spmm_backward": (_I32, [C.POINTER(RoskoPacked), C.POINTER(RoskoPacked), _P, _I64,
                                   _P, _I64, _I64, _P, _I64, _P, _I64, _P, _SZ, _P]),
    "rosko_scatter_dense": (_I32, [C.POINTER(RoskoPacked), _P, _I64, _P, _I64, _P]),
    "rosko_features_workspace_size": (_I32, [_I64, _I64, C.POINTER(_SZ)]),
    "rosko_features": (_I32, [_P, _I64, _I64, _I64, _I64, _P, _SZ, _P, _P]),
    "rosko_mlp_param_count": (_I32, [_I32, _I32, _I32, C.POINTER(_I64)]),
    "rosko_mlp_normalize": (_I32, [_P, _I64, _I32, _P, _P, _P, _P]),
    "rosko_mlp_forward": (_I32, [_P, _I32, _I32, _I32, _P, _I64, _P, _P, _P, _P]),
    "rosko_mlp_backward": (_I32, [_P, _I32, _I32, _I32, _P, _P, _P, _P, _P, _P, _I64, _P, _P,
                                  _P, _P]),
    "rosko_adam_step": (_I32, [_P, _P, _P, _P, _I64, C.c_float, C.c_float, C.c_float,
                               C.c_float, _I32, _P]),
    "rosko_argmin_rows": (_I32, [_P, _I64, _I32, _P, _P]),
    "rosko_sched_candidate": (_I32, [_I32, C.POINTER(_I32), C.POINTER(RoskoPlan)]),
    "rosko_sched_analytic": (_I32, [_P, C.POINTER(_I32)]),
    "rosko_sched_precision": (_I32, [_P, _I32, _I32, C.POINTER(_I32)]),
    "rosko_plan_select": (_I32, [_P, _P, _P, _P, _I32, _I32, C.POINTER(_I32), C.POINTER(_I32),
                                 C.POINTER(RoskoPlan)]),
    "rosko_status_str": (C.c_char_p, [_I32]),
    "rosko_last_error": (C.c_char_p, []),
    "rosko_abi_version": (_I32, []),
}


def lib():
    """Load librosko.so (built by paper_2307_03930_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python paper_2307_03930_amd/build.py` "
                "(or __graft_entry__.build()).  There is no non-HIP fallback.")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != ROSKO_OK:
        msg = lib().rosko_last_error().decode(errors="replace")
        raise RoskoError(status, msg)
