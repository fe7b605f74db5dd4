"""The packer's ways of enqueueing Alg. 1's running offsets (Sec. 4.1) give
the same packed arrays, bit for bit against the oracle:

- two_pass: the count pass, then the write pass;
- auto: one launch whose tiles count their own columns, publish their totals
  and add up those of the tiles before them;
- recount: one launch in which no tile publishes, so every tile counts all
  tiles before it from A itself (the path a tile takes for one whose totals
  have not appeared).

The shapes cover every single-pass tile form: one (panel, column) pair per
lane with panels of up to 8, 16 and 32 rows, two and four pairs per lane, the
record-table staging (more than 1024 tiles), ragged last panels and a
one-tile grid.  A pack captured into a HIP graph takes the two-pass form
(a replay would repeat the launch's tag) and is checked on every replay with
a new matrix."""
import ctypes as C
import dataclasses

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
    """Synchronises; P with the counts of the last pack into its buffers (its
    capacities stay those it was allocated with)."""
    st = P.struct()
    L.check(L.lib().rosko_pack_result(ws.data_ptr(), ws.numel(), C.byref(st),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return dataclasses.replace(P, nnz=int(st.nnz), ncols=int(st.ncols), nrec=int(st.nrec))


def _tiles(M, K, mr):
    P = -(-M // mr)
    pairs = P * K
    cpl = 1 if (mr > 16 or pairs <= 1280 * 64) else (4 if mr <= 8 else 2)
    return -(-pairs // (64 * cpl)), cpl


CASES = [
    (256, 2304, 8, 0.1, "iid"),             # 1152 one-pair tiles: record table
    (256, 2304, 16, 0.3, "iid"),            # 576 one-pair tiles of 16 rows
    (256, 2304, 32, 0.05, "row_clustered"),  # 288 tiles of 32 rows
    (512, 2304, 8, 0.2, "row_clustered"),   # four pairs per lane
    (1024, 2304, 16, 0.05, "column_banded"),  # two pairs per lane, 1152 tiles
    (1024, 4096, 8, 0.05, "iid"),           # four pairs per lane, 2048 tiles (the limit)
    (77, 131, 3, 0.3, "iid"),               # ragged panels of 3 rows
    (100, 70, 24, 0.5, "iid"),              # 24-row panels, ragged last panel
    (37, 1000, 12, 0.1, "iid"),             # 12-row panels
    (5, 5, 1, 0.6, "iid"),                  # one tile
]


@pytest.mark.parametrize("case", CASES)
def test_pack_modes_bit_exact(case):
    M, K, mr, d, kind = case
    tiles, cpl = _tiles(M, K, mr)
    assert tiles <= 2048            # every case takes the single pass in auto
    A = synth.sparse_matrix(M, K, d, 1300 + M + K + mr, kind)
    Ad = dev(A)
    try:
        for dtype in ("f32", "bf16", "fp8"):
            ref = O.pack(A, mr, DT[dtype])
            for mode in ("two_pass", "auto", "recount"):
                say(f"pack {M}x{K} mr={mr} ({tiles} tiles, {cpl} per lane) {dtype} {mode}")
                ops.set_pack_mode(mode)
                assert_pack_equal(ops.pack(Ad, mr, dtype), ref)
    finally:
        ops.set_pack_mode("auto")


def test_repack_into_same_workspace_alternating_modes():
    """Re-packs of changing matrices into one set of buffers and one
    workspace, the single pass after the two-pass form and after itself: the
    words an earlier launch left in the workspace are never taken."""
    M, K, mr = 256, 2304, 16
    A0 = synth.sparse_matrix(M, K, 0.35, 1400, "iid")
    P = ops.pack(dev(A0), mr, "f32")
    ws = torch.empty(max(ops.workspace_size(M, K, mr), 1), dtype=torch.uint8, device="cuda")
    try:
        for step, mode in enumerate(("auto", "auto", "two_pass", "auto", "recount", "auto")):
            # sparser each step, so the capacities of A0's pack always suffice
            A = synth.sparse_matrix(M, K, 0.3 - 0.04 * step, 1401 + step, "iid")
            say(f"repack step {step} {mode}")
            ops.set_pack_mode(mode)
            ops.pack_into(dev(A), P, ws)
            assert_pack_equal(_result(P, ws), O.pack(A, mr, O.F32))
    finally:
        ops.set_pack_mode("auto")


def test_pack_captured_in_graph_replays():
    """A pack captured into a HIP graph, replayed with a different matrix in
    the input buffer each time (the program's own eager work and
    synchronisations between the replays): every replay's arrays against
    the oracle."""
    M, K, mr = 256, 2304, 16
    A0 = synth.sparse_matrix(M, K, 0.3, 1500, "iid")
    Ad = dev(A0)
    P = ops.pack(Ad, mr, "f32")
    ws = torch.empty(max(ops.workspace_size(M, K, mr), 1), dtype=torch.uint8, device="cuda")
    say("pack graph capture")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.pack_into(Ad, P, ws)          # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.pack_into(Ad, P, ws)
    torch.cuda.synchronize()
    for rep in range(4):
        A = synth.sparse_matrix(M, K, 0.28 - 0.05 * rep, 1501 + rep, "iid")
        Ad.copy_(dev(A))
        torch.cuda.synchronize()
        say(f"pack graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert_pack_equal(_result(P, ws), O.pack(A, mr, O.F32))
