"""Host logic of bench.py: the guard that reports the committed HBM traffic
counters only for the SpMM sources they were taken on, and the algorithmic
byte count the HBM fraction is priced against."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _sources(bench):
    d = os.path.join(ROOT, "paper_2307_03930_amd", "csrc")
    out = {}
    for name in bench.SPMM_SOURCES:
        with open(os.path.join(d, name)) as f:
            out[name] = f.read()
    return out


def test_digest_ignores_comments_and_layout(bench):
    src = _sources(bench)
    base = bench.spmm_sources_digest(lambda n: src[n])
    assert base == bench.spmm_sources_digest()
    noisy = dict(src)
    name = bench.SPMM_SOURCES[2]
    noisy[name] = "// a comment\n/* a block\n comment */\n" + src[name].replace(" ", "  ")
    assert bench.spmm_sources_digest(lambda n: noisy[n]) == base


def test_digest_changes_with_code(bench):
    src = _sources(bench)
    base = bench.spmm_sources_digest(lambda n: src[n])
    for name in bench.SPMM_SOURCES:
        changed = dict(src)
        changed[name] = src[name] + "\nstatic int extra_symbol;\n"
        assert bench.spmm_sources_digest(lambda n: changed[n]) != base, name


def test_traffic_reported_only_for_matching_sources(bench, tmp_path, monkeypatch):
    good = tmp_path / "good.txt"
    good.write_text("title line\n  indented: ignored\n"
                    f"sources_sha256: {bench.spmm_sources_digest()}\n"
                    "traffic_bytes_six_calls: 123456789\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(good))
    assert bench.measured_traffic() == 123456789
    stale = tmp_path / "stale.txt"
    stale.write_text("sources_sha256: " + "0" * 64 + "\ntraffic_bytes_six_calls: 123456789\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None


def test_committed_summary_parses(bench):
    with open(bench.PMC_SUMMARY) as f:
        kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    assert len(kv["sources_sha256"].strip()) == 64
    assert int(kv["traffic_bytes_six_calls"].strip()) > 0


def test_alg_bytes_closed_form(bench):
    """Values and row bytes, 8 bytes per kept column, 12 per panel pointer,
    the touched rows of B, and C written (read as well with beta = 1)."""
    nnz, ncols, P, kt, N, M = 1000, 300, 16, 250, 3136, 256
    want = nnz * 5 + ncols * 8 + (P + 1) * 12 + kt * N * 4 + M * N * 4
    assert bench.alg_bytes(nnz, ncols, P, kt, N, M) == want
    assert bench.alg_bytes(nnz, ncols, P, kt, N, M, beta=1) == want + M * N * 4
    assert bench.alg_bytes(nnz, ncols, P, kt, N, M, s_val=1, s_b=2) == \
        nnz * 2 + ncols * 8 + (P + 1) * 12 + kt * N * 2 + M * N * 4
