"""The scheduler's committed timing data and network, checked on the host.

The random-shape corpus (sched_data/corpus.jsonl, 2000 seeded problems)
holds per problem the statistics the GPU computed and the measured SpMM and
repack times of all seven candidates (problems 0..1799 train, 1800..1999
are held out).  The benchmark-shape sweep (measured.jsonl) holds
the same for the six sparse candidates on host-generated matrices, whose
statistics can be checked against the FP64 oracle.  These tests check both
files against their generators, the network's shape, the held-out figures of
the training report (the analytic rule's recomputed through the library, the
network's recomputed through the host forward pass of rosko_plan_select),
and that the network strictly beats the rule it replaces."""
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
        assert r["candidates"] == [0, 1, 2, 3, 4, 5, 6]
        assert len(r["times_us"]) == 7 and min(r["times_us"]) > 0
        assert len(r["pack_us"]) == 7 and min(r["pack_us"]) > 0
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
    assert (Fi, H, Cn) == (16, 64, 7)
    assert len(w["params"]) == Fi * H + H + H * H + H + H * Cn + Cn
    assert len(w["mu"]) == Fi and len(w["sigma"]) == Fi and min(w["sigma"]) > 0
    assert np.isfinite(np.array(w["params"])).all()
    assert w["objective"] in sched.OBJECTIVES


def _corpus():
    with open(os.path.join(DATA, "corpus.jsonl")) as f:
        return sorted((json.loads(line) for line in f if line.strip()), key=lambda r: r["i"])


def test_corpus_covers_the_generator():
    rows = _corpus()
    assert [r["i"] for r in rows] == list(range(2000))
    for r in rows:
        sp = synth.corpus_spec(r["i"])
        for k in ("M", "K", "N", "sparsity", "kind"):
            assert r[k] == sp[k], (r["i"], k)
        assert len(r["times_us"]) == 7 and min(r["times_us"]) > 0
        assert len(r["pack_us"]) == 7 and min(r["pack_us"]) > 0
        assert len(r["features"]) == OF.NFEAT
        assert r["features"][2] == pytest.approx(np.log2(r["N"]), abs=1e-6)


def _times(r, objective):
    t = np.array(r["times_us"])
    return t + np.array(r["pack_us"]) if objective == "step" else t


def _numpy_forward(w, f):
    """The network's forward pass in FP64 (numpy), for the host check."""
    Fi, H, Cn = w["F"], w["H"], w["C"]
    p = np.array(w["params"], np.float64)
    W1 = p[:Fi * H].reshape(Fi, H); o = Fi * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H * Cn].reshape(H, Cn); o += H * Cn
    b3 = p[o:o + Cn]
    x = (np.asarray(f, np.float64) - np.array(w["mu"])) / np.array(w["sigma"])
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3


def test_report_figures_match_library_rule_and_host_network():
    """The held-out slowdowns recorded at training time are what
    rosko_sched_analytic and the host forward pass of rosko_plan_select give
    on the stored statistics; the network strictly beats the analytic rule
    and the best fixed candidate; plan_select agrees with an FP64 numpy
    forward pass wherever the network's two best scores are not a near tie."""
    rows = [r for r in _corpus() if r["i"] >= sched.N_TRAIN]
    with open(os.path.join(DATA, "fit_report.json")) as f:
        rep = json.load(f)
    with open(sched.WEIGHTS) as f:
        w = json.load(f)
    assert rep["data"] == "corpus+sweep" and rep["objective"] == w["objective"]
    assert rep["n_held_out"] == len(rows) == 200
    ana, net = [], []
    for r in rows:
        t = _times(r, rep["objective"])
        ia = sched.plan_select(r["features"], None)[0]
        assert ia == sched.analytic(r["features"])
        ana.append(t[ia] / t.min())
        i, mr, plan = sched.plan_select(r["features"], w)
        net.append(t[i] / t.min())
        y = _numpy_forward(w, r["features"])
        srt = np.sort(y)
        if srt[1] - srt[0] > 1e-4:
            assert i == int(np.argmin(y))
        assert (mr, plan.path) == (sched.candidate(i)[0], sched.candidate(i)[1].path)
    ga = float(np.exp(np.log(ana).mean()))
    gn = float(np.exp(np.log(net).mean()))
    assert ga == pytest.approx(rep["held_out"]["analytic"]["geomean"], rel=1e-9)
    assert gn == pytest.approx(rep["held_out"]["mlp"]["geomean"], rel=2e-3)
    assert rep["held_out"]["mlp"]["geomean"] < rep["held_out"]["analytic"]["geomean"]
    assert rep["held_out"]["mlp"]["geomean"] < rep["held_out"]["best_fixed"]["geomean"]
