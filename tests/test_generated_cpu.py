"""The committed record-loop include matches what its generator writes."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_03930_amd", "csrc")


def test_spmm_loop_include_is_current():
    spec = importlib.util.spec_from_file_location("gen_spmm_loop",
                                                  os.path.join(CSRC, "gen_spmm_loop.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    with open(os.path.join(CSRC, "spmm_loop.inc")) as f:
        assert f.read() == gen.generate(), "run paper_2307_03930_amd/csrc/gen_spmm_loop.py"
