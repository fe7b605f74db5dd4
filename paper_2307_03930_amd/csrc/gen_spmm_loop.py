"""Writes spmm_loop.inc: the record loop of the row-skipping SpMM (Alg. 2)
as one inline-asm block per (register tile, B dtype, pipeline depth).

Why generated: the loop keeps D columns' B rows and 2D column records in
flight with vector loads and waits for each with an exact vmcnt.  Written as
C++ the compiler's wait-count analysis falls back to vmcnt(0) at the head of
the unrolled loop, draining the pipeline every few columns; a single asm
block owns every load it issues and waits for all of them before it ends, so
no load is ever in flight outside the block.

Register plan inside the block (listed as clobbers / pinned operands), for
depth D (4 or 8):
  v0 .. v(2D-1)        column records, slot u holds record i with i % 2D == u
                       (lane l holds dword l & 15 of the 16-dword record)
  next D * W VGPRs     B row units, slot s = i % D (W dwords per unit)
  next V VGPRs         BF16 units widened to FP32 (BF16 B only)
  tile                 from the next multiple of 8: column j of row r at
                       base + j*MR + r
Per column: the header (k << 8 | count) is read with v_readfirstlane,
min(k, K-1) * ldb * elem becomes the SGPR offset of a buffer load of the B
row.  When the column's turn comes, its three row words go to SGPRs
(v_readlane, bytes masked to the tile height) and one computed jump
(s_getpc / s_setpc) enters a run of twelve equal-sized value blocks at the
block of value count-1, so the values are applied without a branch per
value; the count is clamped to [1, 12] first, so the target is always a
block start.  A value block extracts its row byte (s_bfe_u32) into the
index of VGPR-relative addressing (s_set_gpr_idx_idx, SRC2 and DST turned on
once per column) and issues V v_fmac_f32 whose A operand is the value's
lane of the record register broadcast by DPP row_newbcast.  A CPU test
disassembles the build and checks the block spacing the jump assumes.

Run `python gen_spmm_loop.py` after changing it; a CPU test checks that the
committed spmm_loop.inc matches.
"""
import os

TILES = [(8, 4), (16, 4), (32, 2), (32, 4), (64, 2), (128, 1)]
DTYPES = ["f32", "bf16"]
DEPTHS = [4, 8]
PC = 88          # s[88:89]: jump base, s[90:91]: per-record target (both clobbered)


def unit_dwords(dt, v):
    return v if dt == "f32" else max(1, v // 2)


class Plan:
    """Register plan of one variant."""

    def __init__(self, mr, v, dt, D):
        self.mr, self.v, self.dt, self.D = mr, v, dt, D
        self.R = 2 * D
        self.w = unit_dwords(dt, v)
        self.b0 = self.R                       # first B unit register
        nxt = self.b0 + D * self.w
        self.conv0 = nxt if dt == "bf16" else None
        if dt == "bf16":
            nxt += v
        self.nclob = nxt                       # v0 .. v(nclob-1) clobbered
        self.base = (nxt + 7) // 8 * 8         # tile base
        self.nt = mr * v // 32
        # bytes of one value block: s_bfe_u32 with literal (8), s_set_gpr_idx_idx
        # (4), V v_fmac_f32_dpp (8 each)
        self.blk = 12 + 8 * v

    def tile_ranges(self):
        return [(self.base + 32 * q, self.base + 32 * q + 31) for q in range(self.nt)]

    def b_slot(self, s):
        """(load destination text, per-element FP32 register names, conversion asm)."""
        lo = self.b0 + self.w * s
        dst = f"v[{lo}:{lo + self.w - 1}]" if self.w > 1 else f"v{lo}"
        if self.dt == "f32":
            return dst, [f"v{lo + j}" for j in range(self.v)], []
        c = self.conv0
        if self.v == 4:
            conv = [f"v_lshlrev_b32 v{c}, 16, v{lo}", f"v_and_b32 v{c + 1}, 0xffff0000, v{lo}",
                    f"v_lshlrev_b32 v{c + 2}, 16, v{lo + 1}",
                    f"v_and_b32 v{c + 3}, 0xffff0000, v{lo + 1}"]
        elif self.v == 2:
            conv = [f"v_lshlrev_b32 v{c}, 16, v{lo}", f"v_and_b32 v{c + 1}, 0xffff0000, v{lo}"]
        else:
            conv = [f"v_lshlrev_b32 v{c}, 16, v{lo}"]
        return dst, [f"v{c + j}" for j in range(self.v)], conv

    def b_load_op(self):
        nbytes = self.v * (4 if self.dt == "f32" else 2)
        return {16: "buffer_load_dwordx4", 8: "buffer_load_dwordx2", 4: "buffer_load_dword",
                2: "buffer_load_ushort"}[nbytes]

    def fn(self):
        return f"rk_loop_{self.mr}x{self.v}_{self.dt}_d{self.D}"


def gen_variant(mr, v, dt, D):
    pl = Plan(mr, v, dt, D)
    R = pl.R
    bits = mr.bit_length() - 1               # row index width: log2 of the tile height
    cols = [pl.base + j * mr for j in range(v)]
    L = []

    def a(x):
        L.append(x)

    def rload(u):
        # record at the lane offset vro (the run's next record, clamped to its
        # last one), then vro moves on one record (again clamped)
        a(f"buffer_load_dword v{u}, %[vro], %[rr], 0 offen")
        a("v_add_u32 %[vro], 64, %[vro]")
        a("v_min_u32 %[vro], %[vro], %[vlast]")

    def bload(h, s):
        dst, _, _ = pl.b_slot(s)
        a(f"s_lshr_b32 %[k], %[{h}], 8")
        a("s_min_u32 %[k], %[k], %[km1]")        # keeps every B access in bounds
        a("s_mul_i32 %[k], %[k], %[ldbb]")
        a(f"{pl.b_load_op()} {dst}, %[vbo], %[rb], %[k] offen")

    def body(u):
        s = u % D
        dst, bregs, conv = pl.b_slot(s)
        vr = f"v{u}"
        # count of record i (4 bits), then the header of record i+D into the
        # same SGPR (its B row is issued after the values, when slot s is free)
        a(f"s_and_b32 %[c], %[h{s}], 0xf")
        a(f"v_readfirstlane_b32 %[h{s}], v{(u + D) % R}")
        for c in conv:
            a(c)
        for wd in range(3):
            a(f"v_readlane_b32 %[w{wd}], {vr}, {wd + 1}")
        # the jump of record i, interleaved with the B-row offset of record
        # i+D (row clamped to K-1): target = .Le_u - count * block, reached
        # from the base address taken once before the loop.  Counts 13..15
        # (never written by packing) land in padding blocks of s_nop.
        a(f"s_lshr_b32 %[k], %[h{s}], 8")
        a(f"s_mul_i32 %[c], %[c], {pl.blk}")
        a("s_min_u32 %[k], %[k], %[km1]")
        a(f"s_sub_u32 %[c], .Le{u}_%= - .Lbase%=, %[c]")
        a("s_mul_i32 %[k], %[k], %[ldbb]")
        a("s_set_gpr_idx_on %[c], gpr_idx(SRC2,DST)")
        # nothing between the add and its carry: SCC carries the high word
        a(f"s_add_u32 s{PC + 2}, s{PC}, %[c]")
        a(f"s_addc_u32 s{PC + 3}, s{PC + 1}, 0")
        a(f"s_setpc_b64 s[{PC + 2}:{PC + 3}]")
        for _ in range(3 * pl.blk // 4):      # counts 15, 14, 13: three blocks of s_nop
            a("s_nop 0")
        for t in range(11, -1, -1):
            # row byte t, cut to log2(MR) bits: always inside the tile
            a(f"s_bfe_u32 %[x], %[w{t // 4}], {hex((bits << 16) | 8 * (t % 4))}")
            a("s_set_gpr_idx_idx %[x]")
            for j in range(v):
                a(f"v_fmac_f32_dpp v{cols[j]}, {vr}, {bregs[j]} row_newbcast:{4 + t} "
                  "row_mask:0xf bank_mask:0xf")
        L.append(f".Le{u}_%=:")
        a("s_set_gpr_idx_off")
        a(f"{pl.b_load_op()} {dst}, %[vbo], %[rb], %[k] offen")
        rload(u)

    # ---- prologue: the jump base; records 0..D-1, then for each: header,
    # B row, record j+D
    a(f"s_getpc_b64 s[{PC}:{PC + 1}]")
    L.append(".Lbase%=:")
    for j in range(D):
        rload(j)
    for j in range(D):
        a(f"s_waitcnt vmcnt({D - 1 + j})")
        a(f"v_readfirstlane_b32 %[h{j}], v{j}")
        bload(f"h{j}", j)
        rload(D + j)
    a("s_mov_b32 %[nl], %[n]")
    # ---- steady state, unrolled over the 2D record slots.  At the start of
    # step i the loads in flight are, oldest first, B(i) R(i+D) B(i+1) ...
    # B(i+D-1) R(i+2D-1): vmcnt(2D-2) completes B(i) and R(i+D).  nl counts
    # the records left; the borrow of its decrement ends the run.
    a(".Lloop%=:")
    for u in range(R):
        a("s_sub_u32 %[nl], %[nl], 1")
        a("s_cbranch_scc1 .Ldone%=")
        a(f"s_waitcnt vmcnt({2 * D - 2})")
        body(u)
    a("s_branch .Lloop%=")
    a(".Ldone%=:")
    a("s_waitcnt vmcnt(0)")

    text = "".join((f'      "{x}\\n"\n' if x.endswith(":") else f'      "{x}\\n\\t"\n')
                   for x in L)
    outs = ", ".join(f'"+{{v[{lo}:{hi}]}}"(acc.t[{q}])'
                     for q, (lo, hi) in enumerate(pl.tile_ranges()))
    clob = ", ".join(f'"v{r}"' for r in range(pl.nclob))
    hdecl = ", ".join(f"h{j}" for j in range(D))
    houts = ", ".join(f'[h{j}] "=&s"(h{j})' for j in range(D))
    return f"""// {mr} x {v} tile, {dt.upper()} B, {D} B rows in flight; tile at v{pl.base}
__device__ __forceinline__ void {pl.fn()}(Tile<{pl.nt}>& acc, uint32_t n,
                                       __amdgpu_buffer_rsrc_t rr, __amdgpu_buffer_rsrc_t rb,
                                       uint32_t ldbb, uint32_t km1, uint32_t vro0, uint32_t vbo) {{
  uint32_t nl, k, c, x, w0, w1, w2, {hdecl};
  uint32_t vro = vro0;                                // lane offset of the next record
  const uint32_t vlast = vro0 + (n - 1) * 64;         // ... of the run's last record
  asm volatile(
{text}      : {outs}, [vro] "+v"(vro), [nl] "=&s"(nl), [k] "=&s"(k), [c] "=&s"(c), [x] "=&s"(x),
        [w0] "=&s"(w0), [w1] "=&s"(w1), [w2] "=&s"(w2),
        {houts}
      : [n] "s"(n), [ldbb] "s"(ldbb), [km1] "s"(km1), [rr] "s"(rr), [rb] "s"(rb),
        [vlast] "v"(vlast), [vbo] "v"(vbo)
      : {clob}, "s{PC}", "s{PC + 1}", "s{PC + 2}", "s{PC + 3}", "m0", "scc", "memory");
}}
"""


def generate():
    out = ["// Generated by gen_spmm_loop.py -- do not edit.\n"
           "// Record loops of the row-skipping SpMM, one per (tile, B dtype, depth); see the\n"
           "// generator for the register plan and the pipeline.\n"
           "#pragma once\n"]
    for mr, v in TILES:
        for dt in DTYPES:
            for D in DEPTHS:
                out.append(gen_variant(mr, v, dt, D))
    out.append("template <int MR, int V, int TB, int D> struct RkLoop;\n")
    for mr, v in TILES:
        for dt, tb in (("f32", "ROSKO_F32"), ("bf16", "ROSKO_BF16")):
            for D in DEPTHS:
                pl = Plan(mr, v, dt, D)
                out.append(f"""template <> struct RkLoop<{mr}, {v}, {tb}, {D}> {{
  static __device__ __forceinline__ void run(Tile<{pl.nt}>& acc, uint32_t n,
                                             __amdgpu_buffer_rsrc_t rr, __amdgpu_buffer_rsrc_t rb,
                                             uint32_t ldbb, uint32_t km1, uint32_t vro,
                                             uint32_t vbo) {{
    {pl.fn()}(acc, n, rr, rb, ldbb, km1, vro, vbo);
  }}
}};
""")
    return "\n".join(out)


PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spmm_loop.inc")

if __name__ == "__main__":
    with open(PATH, "w") as f:
        f.write(generate())
    print("wrote", PATH)
