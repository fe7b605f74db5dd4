"""Pins of the CPU oracle against things other than itself: the paper's worked
examples, brute force with exact rationals, library routines (numpy matmul,
torch's BF16/FP8 conversions), closed forms and finite differences."""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle as O
from oracle import mlp as OM
from paper_2307_03930_amd import synth
from tests.golden_io import load

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def setup_module(_m):
    O.build(force=True)


# --------------------------------------------------------------------------
# packing: Alg. 1
# --------------------------------------------------------------------------
def _check_golden(name, dtype=O.F32):
    g = load(name)
    pk = O.pack(g["matrix"], g["mr"], dtype)
    np.testing.assert_array_equal(pk.val.astype(np.float64), np.array(g["val"]))
    np.testing.assert_array_equal(pk.loc, np.array(g["loc"], np.uint8))
    np.testing.assert_array_equal(pk.col_ind, np.array(g["col_ind"], np.int32))
    np.testing.assert_array_equal(pk.col_nnz, np.array(g["col_nnz"], np.int32))
    np.testing.assert_array_equal(pk.col_ptr, np.array(g["col_ptr"], np.int64))
    assert pk.nnz == len(g["val"]) and pk.ncols == len(g["col_ind"])


def test_fig5_tile_packs_in_rank_order():
    _check_golden("fig5_tile.txt")


def test_fig4_column_skips_rows_3_and_5():
    _check_golden("fig4_column.txt")


def _numpy_pack(A, mr):
    """Independent route: np.nonzero on each panel's transpose lists the
    stored entries k-major, m ascending, which is the packed order."""
    M, K = A.shape
    val, loc, ci, cn, pnz, pcol = [], [], [], [], [0], [0]
    bits = A.view(np.uint32) & np.uint32(0x7FFFFFFF)
    for r0 in range(0, M, mr):
        panel_bits = bits[r0:r0 + mr]
        ks, ms = np.nonzero(panel_bits.T)
        val.extend(A[r0 + ms, ks].tolist())
        loc.extend(ms.tolist())
        uk, counts = np.unique(ks, return_counts=True)
        ci.extend(uk.tolist())
        cn.extend(counts.tolist())
        pnz.append(len(val))
        pcol.append(len(ci))
    return (np.array(val, np.float32), np.array(loc, np.uint8), np.array(ci, np.int32),
            np.array(cn, np.int32), np.array(pnz, np.int64), np.array(pcol, np.int64))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mr", [1, 3, 8, 16, 32, 64])
def test_pack_matches_numpy_nonzero_route(seed, mr):
    g = synth.rng(100 + seed)
    M, K = int(g.integers(1, 90)), int(g.integers(1, 70))
    A = synth.sparse_matrix(M, K, float(g.uniform(0.02, 0.6)), 200 + seed)
    pk = O.pack(A, mr)
    val, loc, ci, cn, pnz, pcol = _numpy_pack(A, mr)
    assert np.array_equal(pk.val.view(np.uint32), val.view(np.uint32))
    assert np.array_equal(pk.loc, loc)
    assert np.array_equal(pk.col_ind, ci)
    assert np.array_equal(pk.col_nnz, cn)
    assert np.array_equal(pk.panel_nz_ptr, pnz)
    assert np.array_equal(pk.panel_col_ptr, pcol)
    assert np.array_equal(pk.col_ptr, np.concatenate([[0], np.cumsum(cn)]).astype(np.int64))


def test_pack_bit_level_zero_test():
    # -0.0 is skipped; NaN, Inf and subnormals are stored (the structure comes
    # from the bits of the FP32 source).
    A = np.array([[-0.0, np.nan, 1e-45, 0.0],
                  [np.inf, 0.0, -0.0, -2.5]], np.float32)
    pk = O.pack(A, 2)
    assert pk.nnz == 4
    np.testing.assert_array_equal(pk.col_ind, [0, 1, 2, 3])
    np.testing.assert_array_equal(pk.loc, [1, 0, 0, 1])
    assert np.isinf(pk.val[0]) and np.isnan(pk.val[1])
    assert pk.val.view(np.uint32)[2] == 1  # smallest subnormal kept bit-exact


def test_pack_roundtrip_and_invariants():
    for seed in range(5):
        A = synth.sparse_matrix(77, 131, 0.15, 300 + seed, synth.MASK_KINDS[seed % 3])
        for mr in (8, 13, 32):
            pk = O.pack(A, mr)
            assert np.array_equal(O.unpack(pk), A.astype(np.float64))
            bits = A.view(np.uint32) & np.uint32(0x7FFFFFFF)
            assert pk.nnz == int((bits != 0).sum()) == int(pk.col_nnz.sum())
            for p in range(pk.n_panels):
                cs = pk.col_ind[pk.panel_col_ptr[p]:pk.panel_col_ptr[p + 1]]
                assert np.all(np.diff(cs) > 0)
                for c in range(pk.panel_col_ptr[p], pk.panel_col_ptr[p + 1]):
                    lc = pk.loc[pk.col_ptr[c]:pk.col_ptr[c + 1]]
                    assert np.all(np.diff(lc.astype(int)) > 0)
                    assert lc.max() < min(mr, 77 - p * mr)


def test_pack_empty_and_degenerate():
    for shape in [(0, 5), (5, 0), (0, 0), (4, 4)]:
        A = np.zeros(shape, np.float32)
        pk = O.pack(A, 8)
        assert pk.nnz == 0 and pk.ncols == 0
        assert len(pk.panel_nz_ptr) == (shape[0] + 7) // 8 + 1


def test_pack_transpose_equals_pack_of_transposed():
    A = synth.sparse_matrix(40, 23, 0.2, 7)
    pkT = O.pack(np.ascontiguousarray(A.T), 8)
    val, loc, ci, cn, pnz, pcol = _numpy_pack(np.ascontiguousarray(A.T), 8)
    assert np.array_equal(pkT.loc, loc) and np.array_equal(pkT.col_ind, ci)


# --------------------------------------------------------------------------
# value encodings
# --------------------------------------------------------------------------
def _bf16_torch(x):
    return torch.from_numpy(np.array([x], np.float32)).to(torch.bfloat16).view(torch.int16) \
        .numpy().view(np.uint16)[0]


def test_bf16_encode_matches_torch():
    g = synth.rng(11)
    xs = list(g.standard_normal(3000).astype(np.float32) * np.float32(1e3))
    xs += list((g.standard_normal(300) * 1e-39).astype(np.float32))  # subnormals
    # exact ties: low half exactly 0x8000, with odd and even kept parts
    for hi in (0x3F80, 0x3F81, 0xBF80, 0xBF81, 0x0001, 0x7F7F):
        xs.append(np.array([(hi << 16) | 0x8000], np.uint32).view(np.float32)[0])
    xs += [np.float32(x) for x in (0.0, -0.0, np.inf, -np.inf, 3.4028235e38, -3.4028235e38)]
    for x in xs:
        assert O.bf16_encode(float(x)) == int(_bf16_torch(x)), x
    assert O.bf16_encode(float("nan")) == 0x7FC0


def test_bf16_decode_exact():
    for h in (0x0000, 0x3F80, 0xC000, 0x7F80, 0x0001):
        expect = np.array([h << 16], np.uint32).view(np.float32)[0]
        assert O.bf16_decode(h) == expect


def test_fp8_decode_all_codes_match_torch():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    for c in range(256):
        d = O.fp8_decode(c)
        if np.isnan(ref[c]):
            assert np.isnan(d)
        else:
            assert d == ref[c] and np.signbit(d) == np.signbit(ref[c]), c


def test_fp8_encode_matches_torch_in_range():
    g = synth.rng(12)
    ys = list(g.uniform(-464, 464, 4000).astype(np.float32))
    ys += list((g.standard_normal(2000) * 0.01).astype(np.float32))   # subnormal range
    # every midpoint between consecutive finite codes (exact ties)
    vals = sorted({O.fp8_decode(c) for c in range(0x7F)})
    ys += [np.float32((a + b) / 2) for a, b in zip(vals, vals[1:])]
    ys += [np.float32(-(a + b) / 2) for a, b in zip(vals, vals[1:])]
    for y in ys:
        ref = torch.tensor([float(y)], dtype=torch.float32).to(torch.float8_e4m3fn) \
            .view(torch.uint8).item()
        assert O.fp8_encode(float(y)) == ref, y


def test_fp8_encode_saturates():
    for y in (464.1, 500.0, 1e30, float("inf")):
        assert O.fp8_encode(y) == 0x7E
        assert O.fp8_encode(-y) == 0xFE
    assert O.fp8_encode(float("nan")) == 0x7F


def test_row_scale_closed_form():
    A = synth.sparse_matrix(50, 40, 0.3, 13)
    A[3] = 0.0
    s = O.row_scale(A)
    amax = np.abs(A).max(axis=1).astype(np.float32)
    expect = np.where(amax == 0, np.float32(1), amax / np.float32(448))
    assert np.array_equal(s.view(np.uint32), expect.astype(np.float32).view(np.uint32))


def test_fp8_pack_values_decode_within_half_ulp():
    A = synth.sparse_matrix(64, 96, 0.25, 14)
    pk = O.pack(A, 16, O.FP8)
    deq = O.unpack(pk)
    mask = A != 0
    rel = np.abs(deq[mask] - A[mask]) / np.repeat(pk.row_scale, mask.sum(axis=1))
    # rounding error of E4M3 at 3 mantissa bits is at most 2^-4 relative, plus
    # the subnormal floor of 2^-10 in scaled units
    scaled = np.abs(A[mask]) / np.repeat(pk.row_scale, mask.sum(axis=1))
    assert np.all(rel <= np.maximum(scaled * 2.0 ** -4, 2.0 ** -10) * (1 + 1e-6))


# --------------------------------------------------------------------------
# SpMM
# --------------------------------------------------------------------------
def test_spmm_brute_force_exact_rationals():
    g = synth.rng(21)
    for _ in range(8):
        M, K, N = (int(v) for v in g.integers(1, 7, size=3))
        A = (g.integers(-4, 5, size=(M, K)) * (g.random((M, K)) < 0.5)).astype(np.float32)
        B = g.integers(-6, 7, size=(K, N)).astype(np.float32)
        C = O.spmm(A, B)
        for m in range(M):
            for n in range(N):
                exact = sum(Fraction(int(A[m, k])) * Fraction(int(B[k, n])) for k in range(K))
                assert C[m, n] == float(exact)


def test_spmm_hand_case():
    A = np.array([[1, 0, 2], [0, 0, -3]], np.float32)
    B = np.array([[1, 2], [5, 7], [0.5, -1]], np.float32)
    np.testing.assert_array_equal(O.spmm(A, B), [[2.0, 0.0], [-1.5, 3.0]])


def test_spmm_matches_numpy_matmul():
    A = synth.sparse_matrix(70, 150, 0.2, 22)
    B = synth.dense_normal(150, 33, 23)
    C = O.spmm(A, B)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    scale = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)
    assert np.all(np.abs(C - ref) <= 1e-14 * scale + 1e-300)


def test_abs_product_hand_case():
    # (|A| |B|)_i over A's kept entries: row 0 = 1*|B0| + 2*|B2|, row 1 =
    # 3*|B2|; the -0.0 entry is not kept, so the Inf in B's row 1 never meets
    # a zero factor (a dense |A| @ |B| would give NaN there)
    A = np.array([[1, 0, -2], [0, -0.0, -3]], np.float32)
    B = np.array([[1, -2], [np.inf, 7], [0.5, -1]], np.float32)
    np.testing.assert_array_equal(O.abs_product(A, B), [[2.0, 4.0], [1.5, 3.0]])


def test_abs_product_matches_numpy_and_bounds_the_product():
    A = synth.sparse_matrix(60, 140, 0.25, 25)
    B = synth.dense_normal(140, 37, 26)
    S = O.abs_product(A, B)
    ref = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)
    assert np.all(np.abs(S - ref) <= 1e-14 * ref + 1e-300)
    # |sum a b| <= sum |a| |b|, with equality when every term is non-negative
    assert np.all(np.abs(O.spmm(A, B)) <= S * (1 + 1e-14))
    Ap, Bp = np.abs(A), np.abs(B)
    np.testing.assert_array_equal(O.abs_product(Ap, Bp), O.spmm(Ap, Bp))
    # bilinear: scaling B by 2 scales the bound exactly by 2
    np.testing.assert_array_equal(O.abs_product(A, 2 * B), 2 * S)


def test_spmm_csr_rows_hand_case():
    # rows 0 and 2 of a 3 x 3 CSR matrix with an explicit zero in row 0:
    # C[0] = 2*B[1] + 0*B[2], C[2] = -1*B[0] + 4*B[2]
    row_ptr = np.array([0, 2, 2, 4], np.int64)
    col_idx = np.array([1, 2, 2, 0], np.int32)
    val = np.array([2, 0, 4, -1], np.float32)
    B = np.array([[1, 2], [3, -4], [0.5, 8]], np.float32)
    np.testing.assert_array_equal(O.spmm_csr_rows(row_ptr, col_idx, val, B, [0, 2]),
                                  [[6.0, -8.0], [1.0, 30.0]])
    np.testing.assert_array_equal(O.abs_spmm_csr_rows(row_ptr, col_idx, val, B, [2]),
                                  [[3.0, 34.0]])
    np.testing.assert_array_equal(O.spmm_csr_rows(row_ptr, col_idx, val, B, [1]), [[0.0, 0.0]])


def test_spmm_csr_rows_matches_dense_oracle_on_a_graph():
    """On a small power-law graph the CSR definition agrees with the dense
    oracle (a different summation route) to FP64 rounding, and so does the
    absolute-value scale."""
    gr = synth.power_law_graph(600, 12.0, 31)
    A = synth.csr_to_dense(gr)
    B = synth.dense_normal(600, 24, 32)
    rows = list(range(0, 600, 7))
    C = O.spmm_csr_rows(gr.row_ptr, gr.col_idx, gr.val, B, rows)
    S = O.abs_spmm_csr_rows(gr.row_ptr, gr.col_idx, gr.val, B, rows)
    np.testing.assert_allclose(S, O.abs_product(A, B)[rows], rtol=1e-14, atol=0)
    assert np.all(np.abs(C - O.spmm(A, B)[rows]) <= 1e-14 * S + 1e-300)


def test_power_law_graph_structure():
    """The graph generator's output: symmetric, self loops, no repeated
    entries, rows sorted, the GCN normalisation (each value is
    1 / sqrt(d_u d_v)), and the requested mean degree within 3%."""
    gr = synth.power_law_graph(3000, 30.0, 33)
    A = synth.csr_to_dense(gr)
    assert np.array_equal(A != 0, (A != 0).T)
    assert np.all(np.diag(A) > 0)
    d = np.diff(gr.row_ptr)
    for m in range(0, 3000, 97):
        seg = gr.col_idx[gr.row_ptr[m]:gr.row_ptr[m + 1]]
        assert np.all(np.diff(seg) > 0)
    rows = np.repeat(np.arange(3000), d)
    np.testing.assert_allclose(gr.val, 1.0 / np.sqrt(d[rows] * d[gr.col_idx].astype(np.float64)),
                               rtol=1e-6)
    assert abs((gr.nnz - 3000) / 3000 - 30.0) <= 0.9
    assert d.max() > 5 * d.mean()        # heavy tail


def test_conv3x3_direct_hand_case():
    # one input channel 3 x 3 holding 1..9, one output channel; the centre tap
    # (ky = kx = 1) copies the input, the top-left tap (ky = kx = 0) shifts it
    # down-right with zeros entering, so out = X + 2 * shift(X)
    X = np.arange(1, 10, dtype=np.float32).reshape(1, 3, 3)
    A = np.zeros((1, 9), np.float32)
    A[0, 4] = 1.0
    A[0, 0] = 2.0
    want = X[0].astype(np.float64).copy()
    want[1:, 1:] += 2.0 * X[0, :-1, :-1]
    np.testing.assert_array_equal(O.conv3x3_direct(A, X)[0], want)
    # the scale uses |weight| |input|
    np.testing.assert_array_equal(O.conv3x3_direct(-A, -X, absolute=True)[0], want)


def test_conv3x3_direct_equals_im2col_route():
    """The direct definition against the im2col route (im2col then the CSR
    definition of the product), on a pruned layer with ragged sizes."""
    g = synth.rng(41)
    X = np.maximum(g.standard_normal((5, 7, 9)), 0).astype(np.float32)
    A = synth.sparse_matrix(6, 45, 0.3, 42)
    direct = O.conv3x3_direct(A, X)
    via = O.spmm(A, synth.im2col_3x3(X)).reshape(6, 7, 9)
    scale = O.conv3x3_direct(A, X, absolute=True)
    assert np.all(np.abs(direct - via) <= 1e-14 * scale + 1e-300)
    np.testing.assert_array_equal(O.conv3x3_direct(A, X, threads=4), direct)


def test_threaded_oracle_routines_equal_single_thread():
    A = synth.sparse_matrix(70, 90, 0.2, 27)
    B = synth.dense_normal(90, 45, 28)
    dC = synth.dense_normal(70, 45, 29)
    for f in (O.spmm, O.abs_product):
        assert f(A, B, threads=4).tobytes() == f(A, B).tobytes()
    assert O.grad_dB(A, dC, threads=4).tobytes() == O.grad_dB(A, dC).tobytes()
    pk = O.pack(A, 8)
    assert (O.grad_dA_packed(pk, dC, B, threads=4).tobytes()
            == O.grad_dA_packed(pk, dC, B).tobytes())


def test_spmm_csr_equals_dense_bitwise_finite():
    # adding an exact zero product never changes a partial sum that starts at
    # +0, so skipping zero terms is exact (Sec. 3): CSR == dense bit for bit
    A = synth.sparse_matrix(33, 64, 0.3, 24)
    B = synth.dense_normal(64, 17, 25)
    assert np.array_equal(O.spmm(A, B), O.dense_mm(A, B))


def test_spmm_identity_permutation_single():
    B = synth.dense_normal(20, 9, 26)
    assert np.array_equal(O.spmm(np.eye(20, dtype=np.float32), B), B.astype(np.float64))
    perm = synth.rng(27).permutation(20)
    Pm = np.eye(20, dtype=np.float32)[perm]
    assert np.array_equal(O.spmm(Pm, B), B[perm].astype(np.float64))
    S = np.zeros((5, 20), np.float32)
    S[2, 7] = 3.0
    C = O.spmm(S, B)
    assert np.array_equal(C[2], 3.0 * B[7].astype(np.float64))
    assert not C[[0, 1, 3, 4]].any()


def test_spmm_zero_sparsity_equals_dense_numpy():
    A = synth.dense_normal(24, 40, 28)
    B = synth.dense_normal(40, 12, 29)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    scale = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)
    assert O.err_metric(O.spmm(A, B), ref, scale) < 1e-14


@pytest.mark.parametrize("dtype", [O.F32, O.BF16, O.FP8])
@pytest.mark.parametrize("mr", [4, 8, 32])
def test_packed_alg2_route(dtype, mr):
    A = synth.sparse_matrix(45, 70, 0.2, 30)
    B = synth.dense_normal(70, 11, 31)
    pk = O.pack(A, mr, dtype)
    C2 = O.spmm_packed(pk, B)
    # Alg. 2 on the decoded matrix equals the plain product of that matrix
    Adeq = O.unpack(pk)
    ref = Adeq @ B.astype(np.float64)
    scale = np.abs(Adeq) @ np.abs(B).astype(np.float64)
    assert O.err_metric(C2, ref, scale) < 1e-14
    if dtype == O.F32:
        assert np.array_equal(C2, O.spmm(A, B))
    # beta = 1 accumulates onto the given C
    C0 = synth.dense_normal(45, 11, 32).astype(np.float64)
    assert np.allclose(O.spmm_packed(pk, B, C0), C0 + C2, rtol=0, atol=1e-12)


def test_quantised_error_bounds():
    A = synth.sparse_matrix(64, 128, 0.1, 33)
    B = synth.dense_normal(128, 40, 34)
    ref = O.spmm(A, B)
    scale = O.abs_product(A, B)
    e_bf = O.err_metric(O.spmm_packed(O.pack(A, 16, O.BF16), B), ref, scale)
    e_f8 = O.err_metric(O.spmm_packed(O.pack(A, 16, O.FP8), B), ref, scale)
    assert 0 < e_bf <= 2.0 ** -8 * (1 + 1e-9)   # RNE to 8 significant bits: u = 2^-8
    assert 0 < e_f8 <= 2.0 ** -4 * (1 + 1e-9)   # 4 significant bits: u = 2^-4
    # BF16 identity is exact
    I = np.eye(32, dtype=np.float32)
    Bb = synth.bf16_representable(synth.dense_normal(32, 8, 35))
    assert np.array_equal(O.spmm_packed(O.pack(I, 8, O.BF16), Bb), Bb.astype(np.float64))


def test_err_metric_catches_planted_error():
    A = synth.sparse_matrix(10, 12, 0.4, 36)
    B = synth.dense_normal(12, 5, 37)
    ref = O.spmm(A, B)
    scale = O.abs_product(A, B)
    bad = ref.copy()
    bad[3, 2] += 1e-3 * scale[3, 2]
    assert O.err_metric(bad, ref, scale) == pytest.approx(1e-3, rel=1e-6)


# --------------------------------------------------------------------------
# backward
# --------------------------------------------------------------------------
def test_backward_finite_differences_fp64():
    # the loss L = sum(C * G) is bilinear in (A, B), so central differences are
    # exact up to rounding; this checks the gradient routines without using them
    A = synth.sparse_matrix(32, 64, 0.2, 9)
    B = synth.dense_normal(64, 16, 91)
    G = synth.dense_normal(32, 16, 92)
    h = 2.0 ** -10   # a power of two keeps the perturbed FP32 entries exact

    def loss(Ax, Bx):
        return float((O.spmm(Ax, Bx) * G.astype(np.float64)).sum())

    pk = O.pack(A, 8)
    dA = O.grad_dA_packed(pk, G, B)
    dB = O.grad_dB(A, G)
    Aref = O.unpack(pk)
    rows, cols = np.nonzero(Aref)
    # stored entries in packed order
    order = []
    for p in range(pk.n_panels):
        for c in range(pk.panel_col_ptr[p], pk.panel_col_ptr[p + 1]):
            for z in range(pk.col_ptr[c], pk.col_ptr[c + 1]):
                order.append((p * 8 + int(pk.loc[z]), int(pk.col_ind[c])))
    for z, (m, k) in enumerate(order[::7]):
        Ap, Am = A.copy(), A.copy()
        Ap[m, k] += np.float32(h)
        Am[m, k] -= np.float32(h)
        fd = (loss(Ap, B) - loss(Am, B)) / (float(Ap[m, k]) - float(Am[m, k]))
        assert abs(fd - dA[z * 7]) <= 1e-7 * (1 + abs(fd))
    for (k, n) in [(0, 0), (5, 3), (63, 15), (17, 8)]:
        Bp, Bm = B.copy(), B.copy()
        Bp[k, n] += np.float32(h)
        Bm[k, n] -= np.float32(h)
        fd = (loss(A, Bp) - loss(A, Bm)) / (float(Bp[k, n]) - float(Bm[k, n]))
        assert abs(fd - dB[k, n]) <= 1e-7 * (1 + abs(fd))


def test_backward_dense_reference():
    A = synth.sparse_matrix(40, 50, 0.15, 93)
    B = synth.dense_normal(50, 20, 94)
    G = synth.dense_normal(40, 20, 95)
    A64, B64, G64 = (x.astype(np.float64) for x in (A, B, G))
    dB = O.grad_dB(A, G)
    assert np.allclose(dB, A64.T @ G64, rtol=1e-13, atol=1e-13)
    pk = O.pack(A, 16)
    dA = O.grad_dA_packed(pk, G, B)
    dense = (G64 @ B64.T) * (A != 0)
    # scatter the packed-order values back to (m, k)
    back = np.zeros_like(dense)
    for p in range(pk.n_panels):
        for c in range(pk.panel_col_ptr[p], pk.panel_col_ptr[p + 1]):
            for z in range(pk.col_ptr[c], pk.col_ptr[c + 1]):
                back[p * 16 + pk.loc[z], pk.col_ind[c]] = dA[z]
    assert np.allclose(back, dense, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# scheduler MLP
# --------------------------------------------------------------------------
def test_mlp_gradients_finite_differences():
    P = synth.mlp_init_params(5, 7, 3, seed=41)
    P = {k: v.astype(np.float64) for k, v in P.items()}
    P["b1"] = synth.rng(42).standard_normal(7) * 0.1
    X = synth.rng(43).standard_normal((6, 5))
    T = synth.rng(44).standard_normal((6, 3))
    Mk = (synth.rng(45).random((6, 3)) < 0.8).astype(np.float64)
    Y, cache = OM.forward(P, X)
    L, dY = OM.mse_loss(Y, T, Mk)
    g = OM.backward(P, cache, dY)
    h = 1e-6
    for name in OM.PARAM_NAMES:
        flat = P[name].reshape(-1)
        for i in range(0, flat.size, max(1, flat.size // 9)):
            old = flat[i]
            flat[i] = old + h
            Lp = OM.mse_loss(OM.forward(P, X)[0], T, Mk)[0]
            flat[i] = old - h
            Lm = OM.mse_loss(OM.forward(P, X)[0], T, Mk)[0]
            flat[i] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[i]) <= 1e-6 * (1 + abs(fd)), (name, i)


def test_mlp_forward_explicit_loops():
    P = synth.mlp_init_params(3, 4, 2, seed=46)
    X = synth.rng(47).standard_normal((2, 3))
    Y, _ = OM.forward(P, X)
    for b in range(2):
        h1 = [max(0.0, sum(X[b, i] * float(P["W1"][i, j]) for i in range(3)) + float(P["b1"][j]))
              for j in range(4)]
        h2 = [max(0.0, sum(h1[i] * float(P["W2"][i, j]) for i in range(4)) + float(P["b2"][j]))
              for j in range(4)]
        for j in range(2):
            y = sum(h2[i] * float(P["W3"][i, j]) for i in range(4)) + float(P["b3"][j])
            assert abs(y - Y[b, j]) < 1e-12


def test_adam_first_step_closed_form():
    # with bias correction the first step is lr * g / (|g| + eps)
    P = {k: np.ones(3) for k in OM.PARAM_NAMES}
    G = {k: np.array([2.0, -0.5, 1e-3]) for k in OM.PARAM_NAMES}
    Z = {k: np.zeros(3) for k in OM.PARAM_NAMES}
    newp, m, v = OM.adam_step(P, G, Z, Z, t=1, lr=0.1)
    for k in OM.PARAM_NAMES:
        np.testing.assert_allclose(newp[k], 1 - 0.1 * G[k] / (np.abs(G[k]) + 1e-8), rtol=1e-12)
        np.testing.assert_allclose(m[k], 0.1 * G[k], rtol=1e-12)
        np.testing.assert_allclose(v[k], 0.001 * G[k] ** 2, rtol=1e-12)


def test_records_against_independent_rebuild():
    # independent route: rebuild every record from a plain list of
    # (panel, k, row, value) entries made with np.nonzero on each panel
    for seed, mr, dt in ((1, 8, O.F32), (2, 32, O.BF16), (3, 13, O.FP8), (4, 64, O.F32)):
        A = synth.sparse_matrix(70, 700, 0.05 if seed != 4 else 0.4, 900 + seed,
                                "column_banded")
        pk = O.pack(A, mr, dt)
        rec, kb = O.records(pk, 128)
        deq = O.unpack(pk)
        if dt == O.FP8:
            deq = deq / np.repeat(pk.row_scale[:, None], 700, axis=1)
        expect, kbx = [], []
        nkb = (700 + 127) // 128
        for p in range(pk.n_panels):
            panel = A[p * mr:(p + 1) * mr]
            bits = panel.view(np.uint32) & np.uint32(0x7FFFFFFF)
            ks, ms = np.nonzero(bits.T)
            starts = []
            for k in np.unique(ks):
                rows = ms[ks == k]
                for f in range(0, len(rows), 12):
                    part = rows[f:f + 12]
                    d = np.zeros(16, np.uint32)
                    d[0] = (int(k) << 8) | len(part)
                    for t, m in enumerate(part):
                        d[1 + t // 4] |= np.uint32(int(m) << (8 * (t % 4)))
                        d[4 + t] = np.float32(deq[p * mr + m, k]).view(np.uint32)
                    starts.append(int(k))
                    expect.append(d)
            base = len(expect) - len(starts)
            for j in range(nkb + 1):
                kbx.append(base + int(np.searchsorted(np.array(starts, int), j * 128)))
        assert np.array_equal(rec, np.array(expect, np.uint32).reshape(-1, 16))
        assert np.array_equal(kb, np.array(kbx, np.int64))


# --------------------------------------------------------------------------
# scheduler features: hand-derived values on small matrices
# --------------------------------------------------------------------------
def test_features_identity_hand_values():
    from oracle import features as OF
    f = OF.features(np.eye(64, dtype=np.float32), 16)
    # 64 kept values, one per row and per column; each 32-row panel keeps 32
    # of the 64 columns and each 8-row panel 8 of them
    expect = {0: 6.0, 1: 6.0, 2: 4.0, 3: 1 / 64, 5: 0.0, 6: 0.0, 7: 0.0, 8: 0.0,
              9: 1.0, 10: 0.5, 11: 1.0, 12: 0.0, 13: 1.0, 14: np.log2(1 + 64 * 16),
              15: np.log2(64 * 16)}
    for i, v in expect.items():
        assert f[i] == pytest.approx(v, rel=1e-12, abs=1e-15), i
    assert f[4] == pytest.approx(np.log10(1 / 64 + 1e-6))


def test_features_single_value_hand_values():
    from oracle import features as OF
    A = np.zeros((64, 10), np.float32)
    A[40, 3] = -2.5
    f = OF.features(A, 7)
    # rows: one 1 among 64 -> mean 1/64, population variance 1/64 - 1/64^2,
    # CV = sqrt(63); columns: one 1 among 10 -> CV = 3; panels (32 rows):
    # counts [0, 1] -> CV 1, max/mean 2; one kept panel column of 2*10
    assert f[3] == pytest.approx(1 / 640)
    assert f[5] == pytest.approx(np.sqrt(63.0))
    assert f[6] == pytest.approx(63 / 64)
    assert f[7] == pytest.approx(3.0)
    assert f[8] == pytest.approx(0.9)
    assert f[9] == 1.0 and f[11] == 1.0
    assert f[10] == pytest.approx(1 / 20)
    assert f[12] == pytest.approx(1.0) and f[13] == pytest.approx(2.0)
    assert f[14] == pytest.approx(3.0)


def test_features_zero_signs_and_empty():
    from oracle import features as OF
    A = np.full((5, 5), -0.0, np.float32)
    f = OF.features(A, 1)
    assert f[3] == 0.0 and f[4] == pytest.approx(-6.0)
    assert f[6] == 1.0 and f[8] == 1.0 and f[9] == 0.0 and f[13] == 0.0
    A[2, 2] = np.nan
    A[0, 4] = np.float32(1e-45)            # subnormal: kept
    f = OF.features(A, 1)
    assert f[3] == pytest.approx(2 / 25)
    # a 40 x 3 matrix: panels of 32 and 8 rows, last panel short
    B = np.zeros((40, 3), np.float32)
    B[35:40, 1] = 1.0
    B[0, 0] = 1.0
    f = OF.features(B, 2)
    assert f[9] == pytest.approx(6 / 2)      # kept panel columns (32 rows): (0,0), (1,1)
    assert f[11] == pytest.approx(6 / 2)     # (8 rows): panel 0 col 0, panel 4 col 1
    assert f[13] == pytest.approx(5 / 3.0)   # panel counts [1, 5]
