"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/rosko.h declares, and rejects bad arguments on the host with the
documented status codes before any GPU work is enqueued."""
import ctypes as C
import os
import re

import pytest

from paper_2307_03930_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rosko.h")


def setup_module(_m):
    if not os.path.exists(L.LIB_PATH):
        from paper_2307_03930_amd import build
        build.build()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rosko_\w+)\s*\(", text)))


def test_header_declares_expected_calls():
    names = declared_functions()
    for n in ("rosko_pack", "rosko_pack_query", "rosko_pack_transpose", "rosko_spmm",
              "rosko_spmm_backward", "rosko_pack_workspace_size", "rosko_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(L.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(L.SIGNATURES), "binding signatures out of date"


def test_abi_version_and_status_strings():
    lib = L.lib()
    assert lib.rosko_abi_version() == 11
    assert lib.rosko_status_str(L.ROSKO_EINVAL) == b"ROSKO_EINVAL"
    assert lib.rosko_status_str(123) == b"ROSKO_UNKNOWN"


def test_workspace_size_closed_form():
    lib = L.lib()
    n = C.c_size_t(0)
    assert lib.rosko_pack_workspace_size(256, 2304, 32, 0, C.byref(n)) == 0
    P, K = 8, 2304
    NT = (P * K + 63) // 64                 # mr 32: one pair per lane
    r = lambda x: (x + 255) // 256 * 256
    assert n.value == r(4 * P * K) + 2 * r(24 * NT) + r(32)   # tile sums: 3 x int64 per tile
    P2 = (2304 + 31) // 32
    NT2 = (P2 * 256 + 63) // 64
    assert lib.rosko_pack_workspace_size(256, 2304, 8, 0, C.byref(n)) == 0
    P8 = 32                     # mr 8, 73728 pairs: within 1280 one-pair tiles
    NT8 = (P8 * 2304 + 63) // 64
    assert n.value == r(4 * P8 * 2304) + 2 * r(24 * NT8) + r(32)
    assert lib.rosko_pack_workspace_size(1024, 4096, 8, 0, C.byref(n)) == 0
    P8 = 128                    # mr 8, 524288 pairs: four pairs per lane
    NT8 = (P8 * 4096 + 255) // 256
    assert n.value == r(4 * P8 * 4096) + 2 * r(24 * NT8) + r(32)
    assert lib.rosko_pack_workspace_size(1024, 4096, 16, 0, C.byref(n)) == 0
    P16 = 64                    # mr 16, 262144 pairs: two pairs per lane
    NT16 = (P16 * 4096 + 127) // 128
    assert n.value == r(4 * P16 * 4096) + 2 * r(24 * NT16) + r(32)
    assert lib.rosko_pack_workspace_size(256, 2304, 32, 1, C.byref(n)) == 0
    assert n.value == r(4 * P2 * 256) + 2 * r(24 * NT2) + r(32) + r(4 * 256 * 2304)


def test_pack_mode_setting():
    """rosko_pack_set_mode takes the three modes and refuses anything else
    (host only: no GPU call)."""
    lib = L.lib()
    for mode in (L.ROSKO_PACK_TWO_PASS, L.ROSKO_PACK_RECOUNT, L.ROSKO_PACK_AUTO):
        assert lib.rosko_pack_set_mode(mode) == L.ROSKO_OK
    for bad in (-1, 3, 100):
        assert lib.rosko_pack_set_mode(bad) == L.ROSKO_EINVAL
        assert b"mode" in lib.rosko_last_error()
    assert lib.rosko_pack_set_mode(L.ROSKO_PACK_AUTO) == L.ROSKO_OK


@pytest.mark.parametrize("mr", [0, -1, 257])
def test_bad_mr_rejected(mr):
    n = C.c_size_t(0)
    assert L.lib().rosko_pack_workspace_size(10, 10, mr, 0, C.byref(n)) == L.ROSKO_EINVAL
    assert b"mr" in L.lib().rosko_last_error()


def test_query_argument_checks():
    lib = L.lib()
    nnz, nc = C.c_int64(0), C.c_int64(0)
    fake = C.c_void_p(0x1000)   # never dereferenced: every call below fails its checks first
    # negative size
    nr = C.c_int64(0)
    assert lib.rosko_pack_query(fake, -1, 4, 4, 8, fake, 1 << 20, None, C.byref(nnz),
                                C.byref(nc), C.byref(nr)) == L.ROSKO_EINVAL
    # lda < K
    assert lib.rosko_pack_query(fake, 4, 8, 4, 8, fake, 1 << 20, None, C.byref(nnz),
                                C.byref(nc), C.byref(nr)) == L.ROSKO_EINVAL
    # null matrix with nonzero size
    assert lib.rosko_pack_query(None, 4, 4, 4, 8, fake, 1 << 20, None, C.byref(nnz),
                                C.byref(nc), C.byref(nr)) == L.ROSKO_EINVAL
    # workspace too small
    assert lib.rosko_pack_query(fake, 4, 4, 4, 8, fake, 1, None, C.byref(nnz),
                                C.byref(nc), C.byref(nr)) == L.ROSKO_ESMALLBUF
    # null outputs
    assert lib.rosko_pack_query(fake, 4, 4, 4, 8, fake, 1 << 20, None, None,
                                None, None) == L.ROSKO_EINVAL
    # K too wide for the 24-bit column field of the records
    assert lib.rosko_pack_query(fake, 4, 1 << 24, 1 << 24, 8, fake, 1 << 40, None,
                                C.byref(nnz), C.byref(nc), C.byref(nr)) == L.ROSKO_EUNSUPPORTED


def _packed(M, K, mr, dtype=L.ROSKO_F32, fill=True):
    s = L.RoskoPacked()
    s.M, s.K, s.mr, s.n_panels, s.val_dtype = M, K, mr, (M + mr - 1) // mr, dtype
    s.nnz_cap, s.ncols_cap, s.nrec_cap = 10, 10, 10
    if fill:
        for f in ("panel_nz_ptr", "panel_col_ptr", "col_ind", "col_nnz", "col_ptr", "loc",
                  "val", "row_scale", "kblk_ptr", "rec"):
            setattr(s, f, 0x1000)
    return s


def test_pack_argument_checks():
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    s = _packed(8, 8, 4)
    # shape mismatch between arguments and output struct
    assert lib.rosko_pack(fake, 8, 9, 9, 4, L.ROSKO_F32, fake, 1 << 20, C.byref(s),
                          None) == L.ROSKO_EINVAL
    # unsupported value dtype
    assert lib.rosko_pack(fake, 8, 8, 8, 4, 7, fake, 1 << 20, C.byref(s),
                          None) == L.ROSKO_EUNSUPPORTED
    # FP8 without row_scale
    s2 = _packed(8, 8, 4)
    s2.row_scale = None
    assert lib.rosko_pack(fake, 8, 8, 8, 4, L.ROSKO_FP8_E4M3, fake, 1 << 20, C.byref(s2),
                          None) == L.ROSKO_EINVAL
    # null value arrays with nonzero capacity
    s3 = _packed(8, 8, 4)
    s3.val = None
    assert lib.rosko_pack(fake, 8, 8, 8, 4, L.ROSKO_F32, fake, 1 << 20, C.byref(s3),
                          None) == L.ROSKO_EINVAL
    # null record stream
    s5 = _packed(8, 8, 4)
    s5.rec = None
    assert lib.rosko_pack(fake, 8, 8, 8, 4, L.ROSKO_F32, fake, 1 << 20, C.byref(s5),
                          None) == L.ROSKO_EINVAL
    assert b"rec" in lib.rosko_last_error()
    # transpose packing wants the K x M shape
    s4 = _packed(8, 6, 4)
    assert lib.rosko_pack_transpose(fake, 8, 6, 6, 4, L.ROSKO_F32, fake, 1 << 20, C.byref(s4),
                                    None) == L.ROSKO_EINVAL


def test_pack_batch_argument_checks():
    """rosko_pack_batch checks every job before it enqueues anything: a bad
    job, a shared workspace or a shared output is refused on the host."""
    lib = L.lib()
    need = C.c_size_t()
    assert lib.rosko_pack_workspace_size(8, 8, 4, 0, C.byref(need)) == L.ROSKO_OK
    outs = [_packed(8, 8, 4) for _ in range(3)]

    def job(i, ws, ws_bytes=None, out=None, K=8):
        return L.RoskoPackJob(0x1000, 8, K, 8, 4, L.ROSKO_F32, 0, 0, ws,
                              need.value if ws_bytes is None else ws_bytes,
                              C.pointer(out if out is not None else outs[i]))

    def run(js):
        arr = (L.RoskoPackJob * max(len(js), 1))(*js)
        return lib.rosko_pack_batch(len(js), arr, None)

    # batch size and a null job array
    assert lib.rosko_pack_batch(-1, None, None) == L.ROSKO_EINVAL
    assert lib.rosko_pack_batch(L.ROSKO_PACK_BATCH_MAX + 1, None, None) == L.ROSKO_EINVAL
    assert lib.rosko_pack_batch(1, None, None) == L.ROSKO_EINVAL
    # the second job's workspace is too small: its index in the message
    assert run([job(0, 0x100000), job(1, 0x200000, ws_bytes=need.value - 1)]) \
        == L.ROSKO_ESMALLBUF
    assert b"job 1" in lib.rosko_last_error()
    # a job whose shape differs from its output struct
    assert run([job(0, 0x100000), job(1, 0x200000, K=9)]) == L.ROSKO_EINVAL
    # overlapping workspaces (the second starts inside the first)
    assert run([job(0, 0x100000), job(1, 0x100000 + need.value - 256)]) == L.ROSKO_EINVAL
    assert b"workspace" in lib.rosko_last_error()
    # one output struct for two jobs
    assert run([job(0, 0x100000), job(1, 0x200000, out=outs[0])]) == L.ROSKO_EINVAL
    assert b"packed output" in lib.rosko_last_error()
    # a transpose job wants the K x M output and a workspace with the
    # transposed copy: an 8 x 6 A against an 8 x 6 output is refused, and
    # the workspace of a plain 8 x 8 pack is too small for the 8 x 8 transpose
    tj = job(0, 0x100000, out=_packed(8, 6, 4), K=6)
    tj.transpose = 1
    assert run([tj]) == L.ROSKO_EINVAL
    tj = job(0, 0x100000)
    tj.transpose = 1
    assert run([tj]) == L.ROSKO_ESMALLBUF


def test_pack_batch_binding_limits():
    """ops.pack_batch_into refuses more matrices than one call takes before it
    touches any tensor."""
    from paper_2307_03930_amd import ops
    with pytest.raises(ValueError):
        ops.pack_batch_into([None] * (L.ROSKO_PACK_BATCH_MAX + 1))


def test_spmm_argument_checks():
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    s = _packed(8, 8, 4)
    # bad beta, bad ldb/ldc, bad B dtype, wrong n_panels, bad plan tile
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_F32, 16, 16, fake, 16, 2, None,
                          None, 0, None) == L.ROSKO_EINVAL
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_F32, 16, 8, fake, 16, 0, None,
                          None, 0, None) == L.ROSKO_EINVAL
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_F32, 16, 16, fake, 15, 0, None,
                          None, 0, None) == L.ROSKO_EINVAL
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_FP8_E4M3, 16, 16, fake, 16, 0, None,
                          None, 0, None) == L.ROSKO_EUNSUPPORTED
    s.n_panels = 5
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_F32, 16, 16, fake, 16, 0, None,
                          None, 0, None) == L.ROSKO_EINVAL
    s = _packed(8, 8, 4)
    plan = L.RoskoPlan()
    plan.path, plan.cols_per_lane, plan.waves_per_tile, plan.k_split = 5, 4, 2, 1
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_F32, 16, 16, fake, 16, 0, C.byref(plan),
                          None, 0, None) == L.ROSKO_EUNSUPPORTED
    # empty problems are valid no-ops and touch no memory
    s0 = _packed(0, 8, 4)
    assert lib.rosko_spmm(C.byref(s0), fake, L.ROSKO_F32, 16, 16, fake, 16, 0, None,
                          None, 0, None) == L.ROSKO_OK


def test_backward_argument_checks():
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    s = _packed(8, 6, 4)
    st = _packed(8, 6, 4)   # wrong: must be 6 x 8
    assert lib.rosko_spmm_backward(C.byref(s), C.byref(st), fake, 16, fake, 16, 16, fake, 16,
                                   None, 0, None, 0, None) == L.ROSKO_EINVAL
    st = _packed(6, 8, 4, dtype=L.ROSKO_BF16)
    assert lib.rosko_spmm_backward(C.byref(s), C.byref(st), fake, 16, fake, 16, 16, fake, 16,
                                   None, 0, None, 0, None) == L.ROSKO_EUNSUPPORTED
    # a negative dA capacity is rejected before any work
    assert lib.rosko_spmm_backward(C.byref(s), None, fake, 16, fake, 16, 16, None, 16,
                                   fake, -1, None, 0, None) == L.ROSKO_EINVAL


def test_backward_workspace_size():
    """The SDDMM's column-chunk partials: 4 * ceil(N / chunk) * nnz_cap bytes
    when N exceeds one chunk (1024 columns for panels of up to 8 rows, 512 for
    up to 16, 256 for up to 32), none otherwise or for taller panels; with At
    the larger of that and dB's SpMM workspace."""
    lib = L.lib()
    n = C.c_size_t(0)
    for mr, N, want in [(8, 1024, 0), (8, 1025, 4 * 2 * 10), (16, 3136, 4 * 7 * 10),
                        (16, 512, 0), (12, 513, 4 * 2 * 10), (4, 5000, 4 * 5 * 10),
                        (32, 3136, 4 * 13 * 10), (32, 256, 0), (20, 257, 4 * 2 * 10),
                        (64, 3136, 0), (8, 0, 0)]:
        s = _packed(64, 128, mr)
        assert lib.rosko_spmm_backward_workspace_size(C.byref(s), None, N, C.byref(n)) == 0
        assert n.value == want, (mr, N)
    s = _packed(64, 128, 8)
    st = _packed(128, 64, 8)
    assert lib.rosko_spmm_backward_workspace_size(None, C.byref(st), 3136, C.byref(n)) == 0
    only_db = n.value
    assert lib.rosko_spmm_backward_workspace_size(C.byref(s), C.byref(st), 3136,
                                                  C.byref(n)) == 0
    assert n.value == max(only_db, 4 * 4 * 10)
    assert lib.rosko_spmm_backward_workspace_size(C.byref(s), None, -1,
                                                  C.byref(n)) == L.ROSKO_EINVAL
    assert lib.rosko_spmm_backward_workspace_size(None, None, 16, C.byref(n)) == 0
    assert n.value == 0


def test_plan_validation_and_workspace_size():
    lib = L.lib()
    s = _packed(256, 2304, 32)
    n = C.c_size_t(0)
    plan = L.RoskoPlan()
    plan.path, plan.cols_per_lane, plan.waves_per_tile, plan.k_split = 0, 4, 4, 4
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan), C.byref(n)) == 0
    assert n.value == 4 * 4 * 256 * 3136
    plan.k_split = 1000   # clamped to ROSKO_MAX_K_SPLIT
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan), C.byref(n)) == 0
    assert n.value == 4 * 64 * 256 * 3136
    plan.k_split = 1
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan), C.byref(n)) == 0
    assert n.value == 0
    plan.waves_per_tile = 3
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan),
                                         C.byref(n)) == L.ROSKO_EUNSUPPORTED
    # 8 and 16 waves per tile are not offered (their GPU run faulted, cause
    # not found): every tile rejects them
    for mr, V in ((8, 4), (16, 4), (32, 2)):
        s2 = _packed(256, 2304, mr)
        for H in (8, 16):
            plan.cols_per_lane, plan.waves_per_tile = V, H
            st = lib.rosko_spmm_workspace_size(C.byref(s2), 3136, C.byref(plan), C.byref(n))
            assert st == L.ROSKO_EUNSUPPORTED, (mr, V, H)
    plan.cols_per_lane, plan.waves_per_tile = 4, 4
    plan.waves_per_tile, plan.cols_per_lane = 4, 1   # 32 x 1 tile not provided
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan),
                                         C.byref(n)) == L.ROSKO_EUNSUPPORTED
    plan.cols_per_lane, plan.k_split = 4, -1
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan),
                                         C.byref(n)) == L.ROSKO_EINVAL
    plan.waves_per_tile, plan.k_split = 0, 0   # the library chooses both
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, C.byref(plan), C.byref(n)) == 0
    # the automatic plan is valid for every supported panel height
    for mr in (1, 8, 13, 32, 50, 64, 100, 128):
        s2 = _packed(300, 1000, mr)
        assert lib.rosko_spmm_workspace_size(C.byref(s2), 777, None, C.byref(n)) == 0


@pytest.mark.parametrize("mr, nrec, k_split", [
    (16, 16 * 2296, 6),      # long runs (about 2300 records per panel): split, capped by the grid
    (32, 8 * 2550, 4),       # 128-accumulator tiles: 2 wavefronts per SIMD, fewer splits
    (8, 32 * 777, 3),        # 777 records per panel: runs of 64+ records
    (8, 32 * 178, 1),        # short runs: no split, no reduce pass
    (8, 32 * 37, 1),
])
def test_auto_parallel_shape(mr, nrec, k_split):
    """The automatic plan's k_split, read back through the workspace size
    (k_split copies of C, none for 1) on the 256 x 2304 times 3136 layer."""
    lib = L.lib()
    s = _packed(256, 2304, mr)
    s.nrec = nrec
    n = C.c_size_t(0)
    assert lib.rosko_spmm_workspace_size(C.byref(s), 3136, None, C.byref(n)) == 0
    assert n.value == (4 * k_split * 256 * 3136 if k_split > 1 else 0)


@pytest.mark.parametrize("mr, M, N, k_split", [
    (32, 4096, 2048, 3),     # 128 x 8 = 1024 tiles: one wavefront per tile, 3 splits
    (64, 4096, 2048, 3),     # 64 x 16 = 1024 tiles (2 columns per lane)
    (32, 2048, 2048, 6),     # 512 tiles: 3 x 1024 / 512 = 6 splits
    (32, 1024, 2048, 2),     # 256 tiles: 4 wavefronts per tile as before, 2 splits
])
def test_auto_parallel_wide_grid(mr, M, N, k_split):
    """128-accumulator tiles on grids of 512 tiles or more take one
    wavefront per tile and splits filling 3 wavefronts per SIMD (at most 8);
    smaller grids keep the 4-wavefront rule.  4096 columns, about 4000
    records per panel (90% sparsity at mr 32)."""
    lib = L.lib()
    s = _packed(M, 4096, mr)
    s.nrec = s.n_panels * 3958
    n = C.c_size_t(0)
    assert lib.rosko_spmm_workspace_size(C.byref(s), N, None, C.byref(n)) == 0
    assert n.value == 4 * k_split * M * N


def test_sched_candidates_and_analytic_rule():
    lib = L.lib()
    mr = C.c_int32(0)
    plan = L.RoskoPlan()
    seen = []
    for i in range(L.ROSKO_SCHED_CANDIDATES):
        assert lib.rosko_sched_candidate(i, C.byref(mr), C.byref(plan)) == 0
        seen.append((mr.value, plan.path, plan.cols_per_lane))
        assert plan.waves_per_tile == 0 and plan.k_split == 0
    assert seen == [(8, 0, 4), (16, 0, 4), (32, 0, 4), (32, 0, 2), (64, 0, 2), (128, 0, 1),
                    (32, 1, 0)]
    assert lib.rosko_sched_candidate(7, C.byref(mr), C.byref(plan)) == L.ROSKO_EINVAL
    idx = C.c_int32(-1)
    f = (C.c_float * 16)()
    # the rule's table: (density, log2 N) -> candidate
    for d, lN, want in ((0.01, 5.0, 0), (0.01, 10.0, 1), (0.01, 11.5, 3), (0.1, 5.0, 1),
                        (0.1, 10.0, 3), (0.1, 12.0, 3), (0.5, 5.0, 1), (0.5, 10.0, 3),
                        (0.5, 11.0, 6)):
        f[3], f[2] = d, lN
        assert lib.rosko_sched_analytic(f, C.byref(idx)) == 0 and idx.value == want, (d, lN)
        # plan selection without a network is the rule, with the candidate's plan
        i2, m2, p2 = C.c_int32(-1), C.c_int32(0), L.RoskoPlan()
        assert lib.rosko_plan_select(f, None, None, None, L.ROSKO_F32, L.ROSKO_F32,
                                     C.byref(i2), C.byref(m2), C.byref(p2)) == 0
        assert i2.value == want and (m2.value, p2.path, p2.cols_per_lane) == seen[want]
        # the value-type rule: BF16/FP8 values times a BF16 B go dense from
        # density 0.015 up; FP32 operands, or an FP32 B, keep the choice
        for vd, bd in ((L.ROSKO_BF16, L.ROSKO_BF16), (L.ROSKO_FP8_E4M3, L.ROSKO_BF16),
                       (L.ROSKO_F32, L.ROSKO_BF16), (L.ROSKO_BF16, L.ROSKO_F32)):
            assert lib.rosko_plan_select(f, None, None, None, vd, bd, C.byref(i2),
                                         C.byref(m2), C.byref(p2)) == 0
            mfma = vd != L.ROSKO_F32 and bd == L.ROSKO_BF16
            assert i2.value == (6 if mfma and d >= 0.015 else want), (d, lN, vd, bd)
    for d, want in ((0.0149, 1), (0.015, 6), (0.9, 6)):
        f[3], f[2], idx.value = d, 10.0, 1
        assert lib.rosko_sched_precision(f, L.ROSKO_BF16, L.ROSKO_BF16, C.byref(idx)) == 0
        assert idx.value == want
    assert lib.rosko_sched_precision(f, 7, L.ROSKO_BF16, C.byref(idx)) == L.ROSKO_EINVAL
    assert lib.rosko_sched_precision(f, L.ROSKO_BF16, L.ROSKO_FP8_E4M3,
                                     C.byref(idx)) == L.ROSKO_EINVAL
    # a network without its normalisation is refused
    w = (C.c_float * 8000)()
    assert lib.rosko_plan_select(f, w, None, None, L.ROSKO_F32, L.ROSKO_F32, C.byref(i2),
                                 C.byref(m2), C.byref(p2)) == L.ROSKO_EINVAL
    n = C.c_int64(0)
    assert lib.rosko_mlp_param_count(16, 64, 7, C.byref(n)) == 0
    assert n.value == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 7 + 7
    sz = C.c_size_t(0)
    assert lib.rosko_features_workspace_size(100, 50, C.byref(sz)) == 0 and sz.value > 0
    assert lib.rosko_features(None, 0, 5, 5, 3, None, 0, None, None) == L.ROSKO_EINVAL


def test_dense_path_checks_its_workspace_on_the_host():
    """The dense-MFMA path needs the densified A and transposed B in the
    workspace (FP32 size: 4 (Mp + Np) Kp bytes, Mp, Np rounded up to 128 and
    Kp to 64); a smaller one is refused before any work."""
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    s = _packed(8, 8, 4)
    plan = L.RoskoPlan()
    plan.path = L.ROSKO_PATH_DENSE
    n = C.c_size_t(0)
    assert lib.rosko_spmm_workspace_size(C.byref(s), 16, C.byref(plan), C.byref(n)) == 0
    assert n.value == 4 * 128 * 64 + 4 * 128 * 64
    assert lib.rosko_spmm(C.byref(s), fake, L.ROSKO_F32, 16, 16, fake, 16, 0, C.byref(plan),
                          fake, n.value - 1, None) == L.ROSKO_ESMALLBUF
    assert b"dense" in lib.rosko_last_error()


def test_csr_and_row_order_argument_checks():
    """Host-side checks of the CSR packer and the row order, before any
    device work: sizes, limits, null arrays, the dense packers' refusal of
    a row order, an unknown order mode."""
    lib = L.lib()
    fake = C.c_void_p(0x1000)
    n = C.c_size_t(0)
    assert lib.rosko_pack_csr_workspace_size(-1, 4, 0, 8, C.byref(n)) == L.ROSKO_EINVAL
    assert lib.rosko_pack_csr_workspace_size(4, 1 << 24, 0, 8, C.byref(n)) == \
        L.ROSKO_EUNSUPPORTED
    assert lib.rosko_pack_csr_workspace_size(4, 4, 1 << 31, 8, C.byref(n)) == \
        L.ROSKO_EUNSUPPORTED
    assert lib.rosko_pack_csr_workspace_size(4, 4, 0, 0, C.byref(n)) == L.ROSKO_EINVAL
    i64 = C.c_int64(0)
    s = _packed(8, 8, 4)
    assert lib.rosko_pack_csr(None, fake, fake, 8, 8, 3, 4, L.ROSKO_F32, fake, 1 << 20,
                              C.byref(s), None) == L.ROSKO_EINVAL
    assert lib.rosko_pack_csr(fake, None, fake, 8, 8, 3, 4, L.ROSKO_F32, fake, 1 << 20,
                              C.byref(s), None) == L.ROSKO_EINVAL
    assert lib.rosko_pack_csr(fake, fake, fake, 8, 9, 3, 4, L.ROSKO_F32, fake, 1 << 20,
                              C.byref(s), None) == L.ROSKO_EINVAL      # shape mismatch
    assert lib.rosko_pack_csr_query(fake, fake, fake, None, 8, 8, 3, 4, fake, 1 << 20, None,
                                    None, C.byref(i64), C.byref(i64)) == L.ROSKO_EINVAL
    # the dense packers keep the row order
    s.row_perm = 0x1000
    assert lib.rosko_pack(fake, 8, 8, 8, 4, L.ROSKO_F32, fake, 1 << 20, C.byref(s),
                          None) == L.ROSKO_EUNSUPPORTED
    st = _packed(8, 8, 4)
    st.row_perm = 0x1000
    assert lib.rosko_pack_transpose(fake, 8, 8, 8, 4, L.ROSKO_F32, fake, 1 << 20, C.byref(st),
                                    None) == L.ROSKO_EUNSUPPORTED
    assert lib.rosko_row_order(fake, 10, 4, 7, fake, 1 << 20, fake, None) == L.ROSKO_EINVAL
    assert lib.rosko_row_order(fake, 10, 0, 0, fake, 1 << 20, fake, None) == L.ROSKO_EINVAL
    assert lib.rosko_row_order(None, 0, 4, 0, None, 0, None, None) == L.ROSKO_OK
    assert lib.rosko_row_order_workspace_size(0, C.byref(n)) == 0 and n.value == 0
    assert lib.rosko_row_order_workspace_size(-2, C.byref(n)) == L.ROSKO_EINVAL


def test_conv_geometry_and_argument_checks():
    """The padded grid's pitch and copy length, and the direct convolution's
    host-side refusals."""
    lib = L.lib()
    wq, t = C.c_int64(0), C.c_int64(0)
    for (ci, h, w, want_wq) in ((256, 56, 56, 58), (5, 7, 9, 12), (3, 1, 1, 4), (16, 14, 14, 16),
                                (2, 3, 5, 8)):
        assert lib.rosko_conv_geometry(ci, h, w, C.byref(wq), C.byref(t)) == 0
        assert wq.value == want_wq and (h * wq.value) % 4 == 0 and wq.value >= w + 2
        plane = (h + 2) * wq.value
        assert t.value % 4 == 0 and ci * plane + 5 <= t.value <= ci * plane + 11
    assert lib.rosko_conv_geometry(0, 4, 4, C.byref(wq), C.byref(t)) == L.ROSKO_EINVAL
    # 4 T beyond the records' 24-bit column field
    assert lib.rosko_conv_geometry(4096, 64, 64, C.byref(wq), C.byref(t)) == \
        L.ROSKO_EUNSUPPORTED
    fake = C.c_void_p(0x1000)
    s = _packed(8, 45, 4)                   # 9 * 5 columns
    s.nrec = 3
    assert lib.rosko_conv_records(C.byref(s), 4, 7, 9, fake, 10, None) == L.ROSKO_EINVAL
    assert lib.rosko_conv_records(C.byref(s), 5, 7, 9, fake, 2, None) == L.ROSKO_ESMALLBUF
    s.nrec = -1
    assert lib.rosko_conv_records(C.byref(s), 5, 7, 9, fake, 10, None) == L.ROSKO_EINVAL
    plan = L.RoskoPlan()
    plan.path = L.ROSKO_PATH_DENSE
    n = C.c_size_t(0)
    assert lib.rosko_conv_workspace_size(C.byref(s), 7, 9, C.byref(plan), C.byref(n)) == \
        L.ROSKO_EUNSUPPORTED
    assert lib.rosko_conv(C.byref(s), fake, fake, 5, 7, 9, fake, 84, 0, C.byref(plan), None, 0,
                          None) == L.ROSKO_EUNSUPPORTED
    assert lib.rosko_conv(C.byref(s), fake, fake, 5, 7, 9, fake, 83, 0, None, None, 0,
                          None) == L.ROSKO_EINVAL         # ldy < H * Wq = 84
    assert lib.rosko_conv(C.byref(s), fake, fake, 5, 7, 9, fake, 84, 2, None, None, 0,
                          None) == L.ROSKO_EINVAL         # beta
