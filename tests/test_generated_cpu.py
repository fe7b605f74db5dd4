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


# ---------------------------------------------------------------------------
# The record loops enter a run of value blocks through a computed jump whose
# offset is count * (block bytes).  The assembler lays the blocks out; these
# tests read the gfx950 code object of the build back (llvm-objdump of our
# own objects) and check, at every jump site, that the blocks are exactly
# the size the generator multiplies by, that they start right after the
# jump, and that the end label the offset is computed from follows the last
# block.  A mismatch would send a wavefront into the middle of an instruction.
import re
import shutil
import subprocess

import pytest

LLVM = "/opt/rocm/llvm/bin"
_BUILD = os.path.join(ROOT, "paper_2307_03930_amd", "_build")
_INS = re.compile(r"^\s+(\S+)\s*(.*?)\s*//\s*([0-9A-Fa-f]+):")


def _device_disassembly(tu):
    obj = os.path.join(_BUILD, tu + ".o")
    if not os.path.exists(obj):
        from paper_2307_03930_amd import build as B
        B.build()
    tmp = os.path.join(_BUILD, tu + ".check")
    os.makedirs(tmp, exist_ok=True)
    fat, dev = os.path.join(tmp, "fatbin"), os.path.join(tmp, "dev.o")
    subprocess.run([f"{LLVM}/llvm-objcopy", "-O", "binary", "--only-section=.hip_fatbin", obj,
                    fat], check=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o", f"--input={fat}",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={dev}"], check=True)
    out = subprocess.run([f"{LLVM}/llvm-objdump", "-d", dev], check=True, capture_output=True,
                         text=True).stdout
    shutil.rmtree(tmp)
    ins = []
    for line in out.splitlines():
        m = _INS.match(line)
        if m:
            ins.append((int(m.group(3), 16), m.group(1), m.group(2)))
    return ins


@pytest.mark.skipif(not os.path.exists(f"{LLVM}/llvm-objdump"), reason="ROCm LLVM tools missing")
@pytest.mark.parametrize("tu", ["spmm_bf32.hip", "spmm_bbf16.hip"])
def test_record_jump_lands_on_value_blocks(tu):
    """Each loop takes its jump base once (s_getpc_b64 s[88:89] before the
    loop); each column then jumps to base + (END_u - base) - count * BLK with
    the count masked to 4 bits.  Checked at every jump site: the 15 blocks
    (3 of s_nop padding, then values 11..0) are exactly BLK bytes apart and
    start right after the jump, END_u follows the last one, and the add that
    forms the target sits right before its carry and the jump."""
    ins = _device_disassembly(tu)
    sites = [n for n, (_, op, arg) in enumerate(ins) if op == "s_setpc_b64" and "90:91" in arg]
    assert len(sites) > 0
    bases = [n for n, (_, op, arg) in enumerate(ins) if op == "s_getpc_b64" and "88:89" in arg]
    for n in sites:
        assert ins[n - 1][1] == "s_addc_u32" and ins[n - 2][1] == "s_add_u32", ins[n - 3:n + 1]
        base = ins[max(b for b in bases if b < n)][0] + 4        # address after s_getpc_b64
        c = ins[n - 2][2].split(",")[2].strip()
        window = ins[n - 28:n - 2]
        sub = next(x for x in reversed(window)
                   if x[1] == "s_sub_u32" and x[2].split(",")[0].strip() == c)
        mul = next(x for x in reversed(window)
                   if x[1] == "s_mul_i32" and x[2].split(",")[0].strip() == c)
        mask = next(x for x in reversed(window)
                    if x[1] == "s_and_b32" and x[2].split(",")[0].strip() == c)
        assert int(mask[2].split(",")[2].strip(), 0) == 0xF
        blk = int(mul[2].split(",")[2].strip(), 0)
        end = base + int(sub[2].split(",")[1].strip(), 0)
        starts, pad = [], 0
        m = n + 1
        while ins[m][1] != "s_set_gpr_idx_off":
            if ins[m][1] == "s_bfe_u32":
                starts.append(ins[m][0])
            elif ins[m][1] == "s_nop":
                pad += 1
            else:
                assert ins[m][1] in ("s_set_gpr_idx_idx", "v_fmac_f32_dpp"), ins[m]
            m += 1
        assert len(starts) == 12 and pad * 4 == 3 * blk
        assert starts[0] == ins[n][0] + 4 + 3 * blk              # after the jump and padding
        assert all(b - a == blk for a, b in zip(starts, starts[1:]))
        assert end == starts[-1] + blk == ins[m][0]             # s_set_gpr_idx_off at END
        assert end - 15 * blk == ins[n][0] + 4                  # count 15: first padding block
