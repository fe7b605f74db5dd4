"""rosko_pack_batch: several matrices packed in one call, the single passes
of matrices of one kernel form sharing a grid (Alg. 1, Sec. 4.1).  Every
matrix's packed arrays must be those of the oracle, bit for bit, whatever
the batch holds: mixed value types and tile forms, grids too large for the
single pass (packed on their own), more matrices of one form than a launch
takes, every packing mode, and a batch captured into a HIP graph (which
takes the two-pass form) replayed with new matrices."""
import ctypes as C
import dataclasses

import numpy as np
import pytest
import torch

import oracle as O
from paper_2307_03930_amd import _lib as L
from paper_2307_03930_amd import ops, synth
from tests.gpu_helpers import DT, assert_pack_equal, dev, say

pytestmark = pytest.mark.gpu


def setup_module(_m):
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    O.build(force=False)


def teardown_module(_m):
    ops.set_pack_mode("auto")


def _result(P, ws):
    """Synchronises; P with the counts of the last pack into its buffers."""
    st = P.struct()
    L.check(L.lib().rosko_pack_result(ws.data_ptr(), ws.numel(), C.byref(st),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return dataclasses.replace(P, nnz=int(st.nnz), ncols=int(st.ncols), nrec=int(st.nrec))


def _ws(M, K, mr):
    return torch.empty(max(ops.workspace_size(M, K, mr), 1), dtype=torch.uint8, device="cuda")


def _alloc_for(mats, M, K, mr, dtype):
    """Packed buffers whose capacities hold every matrix in mats exactly
    (counts from the oracle; a record holds up to 12 values)."""
    refs = [O.pack(A, mr, DT[dtype]) for A in mats]
    nnz = max(r.nnz for r in refs)
    ncols = max(r.ncols for r in refs)
    nrec = max(int(((r.col_nnz.astype(np.int64) + 11) // 12).sum()) for r in refs)
    return ops._alloc(M, K, mr, ops._dtype_code(dtype), nnz, ncols, nrec, torch.device("cuda"))


def _setup(specs):
    """specs: (M, K, mr, density, kind, dtype, seed); returns (matrices,
    packed buffers sized for them, workspaces)."""
    As, Ps, wss = [], [], []
    for M, K, mr, d, kind, dtype, seed in specs:
        A = synth.sparse_matrix(M, K, d, seed, kind)
        As.append(A)
        Ps.append(_alloc_for([A], M, K, mr, dtype))
        wss.append(_ws(M, K, mr))
    return As, Ps, wss


def _check(specs, As, Ps, wss):
    for (M, K, mr, d, kind, dtype, seed), A, P, ws in zip(specs, As, Ps, wss):
        assert_pack_equal(_result(P, ws), O.pack(A, mr, DT[dtype]))


MIXED = [
    (256, 2304, 16, 0.3, "iid", "f32", 2100),          # 576 one-pair tiles
    (256, 2304, 16, 0.1, "row_clustered", "f32", 2101),  # same form: shares the grid
    (256, 2304, 32, 0.2, "iid", "f32", 2102),          # 288 tiles of 32 rows
    (256, 2304, 8, 0.05, "iid", "f32", 2103),          # 1152 tiles: record table
    (77, 131, 3, 0.3, "iid", "f32", 2104),             # ragged 3-row panels
    (100, 70, 24, 0.5, "iid", "bf16", 2105),           # BF16, ragged last panel
    (37, 1000, 12, 0.1, "iid", "fp8", 2106),           # FP8 with row scales
    (512, 2304, 8, 0.2, "row_clustered", "bf16", 2107),  # four pairs per lane
    (1024, 4096, 8, 0.02, "iid", "f32", 2108),         # 2048 tiles: the largest single pass
    (2048, 4096, 8, 0.02, "iid", "f32", 2109),         # 4096 tiles: packed on its own
    (5, 5, 1, 0.6, "iid", "f32", 2110),                # one tile
]


@pytest.mark.parametrize("mode", ["auto", "two_pass", "recount"])
def test_batch_mixed_bit_exact(mode):
    specs = MIXED if mode != "recount" else [s for s in MIXED if s[0] * s[1] <= 1 << 20]
    As, Ps, wss = _setup(specs)
    try:
        ops.set_pack_mode(mode)
        say(f"pack batch of {len(specs)} mixed matrices, mode {mode}")
        ops.pack_batch_into([(dev(A), P, ws) for A, P, ws in zip(As, Ps, wss)])
        _check(specs, As, Ps, wss)
    finally:
        ops.set_pack_mode("auto")


def test_batch_more_jobs_than_a_launch():
    """Ten matrices of one form: two launches (8 + 2), each matrix exact."""
    specs = [(256, 2304, 16, 0.05 + 0.03 * i, "iid", "f32", 2200 + i) for i in range(10)]
    As, Ps, wss = _setup(specs)
    say("pack batch of 10 same-form matrices")
    ops.pack_batch_into([(dev(A), P, ws) for A, P, ws in zip(As, Ps, wss)])
    _check(specs, As, Ps, wss)


def test_batch_cnn_layer_matches_single_packs():
    """The pruned-CNN layer's six matrices (256 x 2304 at 70 .. 99.8%) with
    panel heights 16, 32, 16, 8, 8, 16: batched, then re-packed one by one
    into the same buffers, and batched again; every pack against the oracle."""
    mrs = [16, 32, 16, 8, 8, 16]
    As = [synth.cnn_weights(s) for s in synth.CNN_SPARSITIES]
    Ps = [ops.pack(dev(A), mr, "f32") for A, mr in zip(As, mrs)]
    wss = [_ws(256, 2304, mr) for mr in mrs]
    refs = [O.pack(A, mr, O.F32) for A, mr in zip(As, mrs)]
    Ads = [dev(A) for A in As]
    for rnd in range(2):
        say(f"cnn layer batch, round {rnd}")
        ops.pack_batch_into(list(zip(Ads, Ps, wss)))
        for P, ws, ref in zip(Ps, wss, refs):
            assert_pack_equal(_result(P, ws), ref)
        for A, P, ws in zip(Ads, Ps, wss):
            ops.pack_into(A, P, ws)
        for P, ws, ref in zip(Ps, wss, refs):
            assert_pack_equal(_result(P, ws), ref)


def test_batch_captured_in_graph_replays():
    """A batch captured into a HIP graph (two-pass form), replayed with new
    matrices in the input buffers, eager work and synchronisations between
    the replays; every replay's arrays against the oracle."""
    specs = [(256, 2304, 16, 0.3, "iid", "f32", 2300), (256, 2304, 8, 0.1, "iid", "f32", 2301),
             (100, 70, 24, 0.5, "iid", "bf16", 2302)]
    firsts = [synth.sparse_matrix(M, K, d, seed, kind) for M, K, mr, d, kind, dtype, seed in specs]
    news = [[synth.sparse_matrix(M, K, d - 0.03 * (rep + 1), seed + 10 * (rep + 1), kind)
             for M, K, mr, d, kind, dtype, seed in specs] for rep in range(3)]
    Ps = [_alloc_for([firsts[i]] + [n[i] for n in news], M, K, mr, dtype)
          for i, (M, K, mr, d, kind, dtype, seed) in enumerate(specs)]
    wss = [_ws(M, K, mr) for M, K, mr, d, kind, dtype, seed in specs]
    Ads = [dev(A) for A in firsts]
    say("pack batch graph capture")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.pack_batch_into(list(zip(Ads, Ps, wss)))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.pack_batch_into(list(zip(Ads, Ps, wss)))
    torch.cuda.synchronize()
    for rep in range(3):
        for Ad, A in zip(Ads, news[rep]):
            Ad.copy_(dev(A))
        torch.cuda.synchronize()
        say(f"pack batch graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        for (M, K, mr, d, kind, dtype, seed), A, P, ws in zip(specs, news[rep], Ps, wss):
            assert_pack_equal(_result(P, ws), O.pack(A, mr, DT[dtype]))


def test_batch_with_transposed_packs():
    """A training step's packs in one call: two weights (256 x 2304 and
    256 x 256 at 90%, mr 8) and their transposes; each against the oracle's
    pack of W and of W^T."""
    mr = 8
    Ws = [synth.sparse_matrix(256, 2304, 0.1, 2400, "iid"),
          synth.sparse_matrix(256, 256, 0.1, 2401, "iid")]
    items, checks = [], []
    for W in Ws:
        M, K = W.shape
        Wd = dev(W)
        P = _alloc_for([W], M, K, mr, "f32")
        Pt = _alloc_for([W.T.copy()], K, M, mr, "f32")
        ws = _ws(M, K, mr)
        ws_t = torch.empty(max(ops.workspace_size(M, K, mr, transpose=True), 1),
                           dtype=torch.uint8, device="cuda")
        items += [(Wd, P, ws), (Wd, Pt, ws_t, True)]
        checks += [(P, ws, O.pack(W, mr, O.F32)), (Pt, ws_t, O.pack(W.T.copy(), mr, O.F32))]
    for rnd in range(2):
        say(f"pack batch with transposes, round {rnd}")
        ops.pack_batch_into(items)
        for P, ws, ref in checks:
            assert_pack_equal(_result(P, ws), ref)


def test_batch_with_empty_matrices():
    """Empty and all-zero matrices in a batch beside a normal one: each gets
    the oracle's empty pointer arrays, the normal one its exact pack."""
    from tests.gpu_helpers import packed_to_np
    mr = 8
    items, empties = [], []
    for shape in [(0, 10), (10, 0), (0, 0), (33, 17)]:
        A = np.zeros(shape, np.float32)
        Ad = dev(A) if A.size else torch.zeros(shape, dtype=torch.float32, device="cuda")
        P = ops.pack(Ad, mr)
        ws = _ws(shape[0], shape[1], mr)
        items.append((Ad, P, ws))
        empties.append((A, P, ws))
    B = synth.sparse_matrix(256, 2304, 0.2, 2500, "iid")
    PB = _alloc_for([B], 256, 2304, mr, "f32")
    wsB = _ws(256, 2304, mr)
    items.insert(2, (dev(B), PB, wsB))
    say("pack batch with empty matrices")
    ops.pack_batch_into(items)
    assert_pack_equal(_result(PB, wsB), O.pack(B, mr, O.F32))
    for A, P, ws in empties:
        R = _result(P, ws)
        ref = O.pack(A, mr)
        assert R.nnz == 0 and R.ncols == 0 and R.nrec == 0
        assert np.array_equal(packed_to_np(R)["panel_nz_ptr"], ref.panel_nz_ptr)
