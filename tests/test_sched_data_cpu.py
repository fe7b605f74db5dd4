"""The scheduler's committed timing data and network, checked on the host.

The measured sweep (sched_data/measured.jsonl) holds, per (matrix, N), the
statistics the GPU computed and the measured SpMM and repack times of the
six sparse candidates.  These tests check that it covers exactly the matrices and N of
the sweep's generator, that its statistics agree with the FP64 oracle on a
sample of matrices regenerated from their seeds, that the committed network
has the shape of the six-candidate scorer, and that the analytic rule's
held-out figure in the training report is what the library's rule gives on
the stored data."""
import ctypes as C
import json
import os

import numpy as np
import pytest

from oracle import features as OF
from paper_2307_03930_amd import _lib as L
from paper_2307_03930_amd import sched, synth

DATA = sched.DATA_DIR


def _rows():
    with open(os.path.join(DATA, "measured.jsonl")) as f:
        return [json.loads(line) for line in f if line.strip()]


def test_measured_sweep_covers_the_generator():
    rows = _rows()
    specs = synth.sweep_specs()
    got = {(r["j"], r["N"]) for r in rows}
    assert got == {(sp["j"], N) for sp in specs for N in synth.SWEEP_N}
    assert len(rows) == len(got)
    for r in rows:
        sp = specs[r["j"]]
        for k in ("M", "K", "sparsity", "kind", "seed", "held_out"):
            assert r[k] == sp[k], (r["j"], k)
        assert r["candidates"] == [0, 1, 2, 3, 4, 5]
        assert len(r["times_us"]) == 6 and min(r["times_us"]) > 0
        assert len(r["pack_us"]) == 6 and min(r["pack_us"]) > 0
        assert len(r["features"]) == OF.NFEAT
        assert r["features"][2] == pytest.approx(np.log2(r["N"]), abs=1e-6)


@pytest.mark.parametrize("j", [50, 62, 67, 79])
def test_stored_statistics_match_oracle(j):
    """Regenerate a 2304 x 256 or 512 x 512 matrix of the sweep from its
    seed and compare the GPU's stored statistics with the oracle's."""
    sp = synth.sweep_specs()[j]
    A = synth.sparse_matrix(sp["M"], sp["K"], 1.0 - sp["sparsity"], sp["seed"], sp["kind"])
    for r in _rows():
        if r["j"] != j:
            continue
        ref = OF.features(A, r["N"])
        np.testing.assert_allclose(np.array(r["features"]), ref, rtol=2e-6, atol=1e-6)


def test_committed_network_shape():
    with open(sched.WEIGHTS) as f:
        w = json.load(f)
    Fi, H, Cn = w["F"], w["H"], w["C"]
    assert (Fi, H, Cn) == (16, 64, 6)
    assert len(w["params"]) == Fi * H + H + H * H + H + H * Cn + Cn
    assert len(w["mu"]) == Fi and len(w["sigma"]) == Fi and min(w["sigma"]) > 0
    assert np.isfinite(np.array(w["params"])).all()
    assert w["objective"] in sched.OBJECTIVES


def test_report_analytic_figure_matches_library_rule():
    """The analytic rule's held-out slowdown recorded at training time is
    what rosko_sched_analytic gives on the stored statistics; the network's
    recorded figure matches it (within 0.5%) and beats the best fixed
    candidate."""
    rows = _rows()
    with open(os.path.join(DATA, "fit_report.json")) as f:
        rep = json.load(f)
    lib = L.lib()
    ratios = []
    n_held = 0
    for r in rows:
        if not r["held_out"]:
            continue
        n_held += 1
        f = np.ascontiguousarray(r["features"], np.float32)
        idx = C.c_int32(-1)
        assert lib.rosko_sched_analytic(f.ctypes.data_as(C.c_void_p), C.byref(idx)) == 0
        t = np.array(r["times_us"])
        if rep["objective"] == "step":
            t = t + np.array(r["pack_us"])
        ratios.append(t[idx.value] / t.min())
    assert rep["n_held_out"] == n_held
    geo = float(np.exp(np.log(ratios).mean()))
    assert geo == pytest.approx(rep["held_out"]["analytic"]["geomean"], rel=1e-9)
    assert rep["held_out"]["mlp"]["geomean"] <= geo * 1.005
    assert rep["held_out"]["mlp"]["geomean"] < rep["held_out"]["best_fixed"]["geomean"]
