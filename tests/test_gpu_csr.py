"""CSR input (graphs) and the inspector's row order on the GPU against the
oracle: the CSR packer must give the packed arrays of Alg. 1 applied to the
row-permuted dense matrix, bit for bit; SpMM and the backward over such a pack
must match the oracle in the matrix's own row order."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import _lib as L
from paper_2307_03930_amd import ops, synth
from tests.gpu_helpers import DT, assert_pack_equal, dev, err, say, threads

pytestmark = pytest.mark.gpu
TOL = 1e-5


def setup_module(_m):
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    O.build(force=False)


def _csr_of(A: np.ndarray, seed: int, extras: bool = True):
    """CSR arrays of A; with extras, each row also stores a few explicit zeros
    (+0.0 and -0.0, which packing drops) and its entries are shuffled."""
    g = synth.rng(seed)
    rows, cols, vals = [], [], []
    for m in range(A.shape[0]):
        nz = np.flatnonzero(A[m].view(np.uint32) & np.uint32(0x7FFFFFFF))
        c = list(nz)
        v = list(A[m, nz])
        if extras and A.shape[1] > 0:
            zero_cols = np.setdiff1d(np.arange(A.shape[1]), nz)
            k = min(len(zero_cols), int(g.integers(0, 3)))
            for z in g.choice(zero_cols, k, replace=False) if k else []:
                c.append(int(z))
                v.append(np.float32(-0.0) if g.random() < 0.5 else np.float32(0.0))
            order = g.permutation(len(c))
            c = [c[i] for i in order]
            v = [v[i] for i in order]
        rows.append(len(c))
        cols += c
        vals += v
    row_ptr = np.zeros(A.shape[0] + 1, np.int64)
    np.cumsum(rows, out=row_ptr[1:])
    return (row_ptr, np.array(cols, np.int32).reshape(-1),
            np.array(vals, np.float32).reshape(-1))


def _perm(kind, row_ptr, mr, seed):
    M = len(row_ptr) - 1
    if kind is None:
        return None
    if kind == "random":
        return synth.rng(seed).permutation(M).astype(np.int32)
    return ops.row_order(dev(row_ptr), mr, kind).cpu().numpy()


def _pack(row_ptr, col, val, K, mr, dtype, perm):
    return ops.pack_csr(dev(row_ptr), dev(col), dev(val), K, mr, dtype,
                        None if perm is None else dev(perm))


CASES = [(37, 300, 0.1, "iid"), (64, 129, 0.3, "row_clustered"), (200, 1000, 0.01, "iid"),
         (96, 257, 0.05, "column_banded"), (9, 5, 0.6, "iid")]


@pytest.mark.parametrize("order", [None, "degree", "balanced", "random"])
@pytest.mark.parametrize("mr", [1, 4, 8, 12, 32, 200])
@pytest.mark.parametrize("case", CASES)
def test_pack_csr_bit_exact(case, mr, order):
    M, K, d, kind = case
    say(f"pack_csr {M}x{K} d={d} {kind} mr={mr} order={order}")
    A = synth.sparse_matrix(M, K, d, 900 + M + K, kind)
    row_ptr, col, val = _csr_of(A, 901 + M)
    perm = _perm(order, row_ptr, mr, 902 + mr)
    Ap = A if perm is None else A[perm]
    for dtype in ("f32", "bf16", "fp8"):
        P = _pack(row_ptr, col, val, K, mr, dtype, perm)
        assert_pack_equal(P, O.pack(Ap, mr, DT[dtype]))


@pytest.mark.parametrize("mr", [8, 16, 64])
def test_pack_csr_power_law_graph(mr):
    """A 4000-node power-law graph (hubs of a few hundred entries among rows of
    a handful), natural and balanced order."""
    gr = synth.power_law_graph(4000, 20.0, 903)
    say(f"pack_csr graph n=4000 nnz={gr.nnz} mr={mr}")
    A = synth.csr_to_dense(gr)
    for order in (None, "balanced"):
        perm = _perm(order, gr.row_ptr, mr, 0)
        P = _pack(gr.row_ptr, gr.col_idx, gr.val, gr.n, mr, "f32", perm)
        assert_pack_equal(P, O.pack(A if perm is None else A[perm], mr, O.F32))


def test_pack_csr_empty_inputs():
    say("pack_csr empty inputs")
    for M, K in ((0, 5), (6, 0), (6, 7)):
        row_ptr = np.zeros(M + 1, np.int64)
        col = np.zeros(0, np.int32)
        val = np.zeros(0, np.float32)
        P = _pack(row_ptr, col, val, K, 4, "f32", None)
        assert_pack_equal(P, O.pack(np.zeros((M, K), np.float32), 4, O.F32))
    # rows holding only explicit zeros
    row_ptr = np.array([0, 2, 2, 3], np.int64)
    P = _pack(row_ptr, np.array([1, 3, 0], np.int32), np.array([0.0, -0.0, 0.0], np.float32),
              4, 2, "f32", None)
    assert P.nnz == 0 and P.ncols == 0


def test_row_order_definitions():
    """degree: rows by descending length, ties by ascending row; balanced:
    the length-sorted rows dealt to the panels in a serpentine, panels
    ascending in even rounds and descending in odd ones (a short last panel
    sits out the rounds beyond its rows)."""
    gr = synth.power_law_graph(1003, 15.0, 904)
    d = np.diff(gr.row_ptr)
    order = np.argsort(-d, kind="stable")
    mr = 8
    say("row order definitions")
    got = ops.row_order(dev(gr.row_ptr), mr, "degree").cpu().numpy()
    np.testing.assert_array_equal(got, order)
    P = -(-1003 // mr)
    last = 1003 - (P - 1) * mr
    want = np.empty(1003, np.int64)
    r = 0
    for q in range(mr):
        panels = list(range(P if q < last else P - 1))
        if q % 2:
            panels.reverse()
        for p in panels:
            want[p * mr + q] = order[r]
            r += 1
    got = ops.row_order(dev(gr.row_ptr), mr, "balanced").cpu().numpy()
    np.testing.assert_array_equal(got, want)
    # balanced panels: their entry counts spread far less than natural order's
    def spread(perm):
        rows = d if perm is None else d[perm]
        pan = np.add.reduceat(rows, np.arange(0, 1003, mr))
        return pan.max() / pan.mean()
    assert spread(got) < spread(None)


@pytest.mark.parametrize("order", [None, "degree", "balanced"])
@pytest.mark.parametrize("mr", [8, 16, 32])
def test_spmm_csr_rows_land_in_matrix_order(mr, order):
    """C = A B from a CSR pack in a row order: every element against the
    oracle in A's own row order, on the sparse path (no K split, a K split
    through the reduce kernel) and the dense-MFMA path, beta 0 and 1."""
    gr = synth.power_law_graph(3000, 25.0, 905)
    A = synth.csr_to_dense(gr)
    B = synth.dense_normal(3000, 96, 906)
    say(f"spmm csr n=3000 mr={mr} order={order}")
    perm = _perm(order, gr.row_ptr, mr, 0)
    P = _pack(gr.row_ptr, gr.col_idx, gr.val, gr.n, mr, "f32", perm)
    ref = O.spmm(A, B)
    scale = O.abs_product(A, B)
    C0 = synth.dense_normal(3000, 96, 907)
    for plan in (ops.make_plan(4, 2, 1), ops.make_plan(4, 4, 3), ops.dense_plan()):
        C = ops.spmm(P, dev(B), plan=plan)
        assert err(C.cpu().numpy(), ref, scale) <= TOL
        Cb = dev(C0)
        ops.spmm(P, dev(B), Cb, beta=1, plan=plan)
        assert err(Cb.cpu().numpy(), ref + C0, scale + np.abs(C0)) <= TOL


@pytest.mark.parametrize("order", [None, "balanced"])
def test_backward_and_scatter_with_row_order(order):
    """dA of C = A B for a CSR pack in a row order: in the pack's order, the
    dot products of dC row perm[i] with B rows; scattered back it is
    (dC B^T) on A's mask in A's own row order."""
    gr = synth.power_law_graph(1500, 20.0, 908)
    A = synth.csr_to_dense(gr)
    B = synth.dense_normal(1500, 1300, 909)      # N over 1024: the chunked SDDMM
    dC = synth.dense_normal(1500, 1300, 910)
    mr = 8
    say(f"backward csr n=1500 order={order}")
    perm = _perm(order, gr.row_ptr, mr, 0)
    P = _pack(gr.row_ptr, gr.col_idx, gr.val, gr.n, mr, "f32", perm)
    dA, _ = ops.spmm_backward(P, None, dev(B), dev(dC), need_dB=False)
    pk = O.pack(A if perm is None else A[perm], mr, O.F32)
    dCp = dC if perm is None else dC[perm]
    ref = O.grad_dA_packed(pk, dCp, B, threads=threads())
    sc = O.grad_dA_packed(pk, np.abs(dCp), np.abs(B), threads=threads())
    assert err(dA.cpu().numpy(), ref, sc) <= TOL
    out = torch.zeros((1500, 1500), dtype=torch.float32, device="cuda")
    ops.scatter_dense(P, dA, out)
    full = (dC.astype(np.float64) @ B.astype(np.float64).T) * (A != 0)
    fsc = (np.abs(dC).astype(np.float64) @ np.abs(B).astype(np.float64).T) * (A != 0)
    assert err(out.cpu().numpy(), full, fsc) <= TOL


def test_pack_csr_rejects_invalid_input():
    """Checks that run on the device: a column twice in a row, a column out
    of range, row pointers out of range, a row order that is not a
    permutation; each makes the query fail with ROSKO_EINVAL."""
    say("pack_csr invalid input")
    ok = (np.array([0, 2, 3], np.int64), np.array([0, 2, 1], np.int32),
          np.array([1.0, 2.0, 3.0], np.float32))
    _pack(*ok, 3, 2, "f32", None)
    bad = [
        (np.array([0, 2, 3], np.int64), np.array([2, 2, 1], np.int32), ok[2], None),
        (np.array([0, 2, 3], np.int64), np.array([0, 3, 1], np.int32), ok[2], None),
        (np.array([0, 2, 4], np.int64), ok[1], ok[2], None),
        (ok[0], ok[1], ok[2], np.array([1, 1], np.int32)),
        (ok[0], ok[1], ok[2], np.array([0, 2], np.int32)),
    ]
    for row_ptr, col, val, perm in bad:
        with pytest.raises(L.RoskoError) as ei:
            _pack(row_ptr, col, val, 3, 2, "f32", perm)
        assert ei.value.status == L.ROSKO_EINVAL


def test_gcn_aggregation_medium_graph_sampled():
    """A 60000-node power-law graph (mean degree 120, 99.8% sparse) times a
    feature matrix of 256 columns, balanced order, mr 16: 600 sampled rows
    against the CSR oracle, and the pack's totals against a host count."""
    gr = synth.power_law_graph(60000, 120.0, 911)
    say(f"gcn medium graph nnz={gr.nnz}")
    X = synth.dense_normal(60000, 256, 912)
    perm = _perm("balanced", gr.row_ptr, 16, 0)
    P = _pack(gr.row_ptr, gr.col_idx, gr.val, gr.n, 16, "f32", perm)
    assert P.nnz == gr.nnz
    rows = np.unique(synth.rng(913).integers(0, 60000, 600))
    C = ops.spmm(P, dev(X)).cpu().numpy()[rows]
    ref = O.spmm_csr_rows(gr.row_ptr, gr.col_idx, gr.val, X, rows)
    sc = O.abs_spmm_csr_rows(gr.row_ptr, gr.col_idx, gr.val, X, rows)
    assert err(C, ref, sc) <= TOL
