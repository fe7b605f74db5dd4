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
row; the values are broadcast from the record register with DPP
row_newbcast into v_fmac_f32 whose accumulator is addressed relative to the
row byte (s_set_gpr_idx_on, SRC2 and DST).

Run `python gen_spmm_loop.py` after changing it; a CPU test checks that the
committed spmm_loop.inc matches.
"""
import os

TILES = [(8, 4), (16, 4), (32, 2), (32, 4), (64, 2), (128, 1)]
DTYPES = ["f32", "bf16"]
DEPTHS = [4, 8]


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
    mask = "0x%08x" % ((mr - 1) * 0x01010101)
    cols = [pl.base + j * mr for j in range(v)]
    L = []

    def a(x):
        L.append(x)

    def rload_const(j):
        a(f"s_min_u32 %[t], {j}, %[nm1]")
        a("s_lshl_b32 %[t], %[t], 6")
        a(f"buffer_load_dword v{j}, %[vro], %[rr], %[t] offen")

    def bload(h, s):
        dst, _, _ = pl.b_slot(s)
        a(f"s_lshr_b32 %[k], %[{h}], 8")
        a("s_min_u32 %[k], %[k], %[km1]")        # keeps every B access in bounds
        a("s_mul_i32 %[k], %[k], %[ldbb]")
        a(f"{pl.b_load_op()} {dst}, %[vbo], %[rb], %[k] offen")

    def body(u):
        s = u % D
        _, bregs, conv = pl.b_slot(s)
        vr = f"v{u}"
        end = f".Lr{u}_%="
        a(f"s_and_b32 %[c], %[h{s}], 0xff")
        for c in conv:
            a(c)
        a("s_nop 1")
        word = 1
        a(f"v_readlane_b32 %[w], {vr}, 1")
        a(f"s_and_b32 %[w], %[w], {mask}")
        for t in range(12):
            if t > 0:
                a(f"s_cmp_lt_u32 %[c], {t + 1}")
                a(f"s_cbranch_scc1 {end}")
                if t % 4 == 0:
                    word += 1
                    a("s_set_gpr_idx_off")
                    a(f"v_readlane_b32 %[w], {vr}, {word}")
                    a(f"s_and_b32 %[w], %[w], {mask}")
                else:
                    a("s_lshr_b32 %[w], %[w], 8")
            a("s_set_gpr_idx_on %[w], gpr_idx(SRC2,DST)")
            for j in range(v):
                a(f"v_fmac_f32_dpp v{cols[j]}, {vr}, {bregs[j]} row_newbcast:{4 + t} "
                  "row_mask:0xf bank_mask:0xf")
        a(f"{end}:")
        a("s_set_gpr_idx_off")

    # ---- prologue: records 0..D-1, then for each: header, B row, record j+D
    a("s_mov_b32 %[i], 0")
    for j in range(D):
        rload_const(j)
    for j in range(D):
        a(f"s_waitcnt vmcnt({D - 1 + j})")
        a(f"v_readfirstlane_b32 %[h{j}], v{j}")
        bload(f"h{j}", j)
        rload_const(D + j)
    # ---- steady state, unrolled over the 2D record slots.  At the start of
    # step i the loads in flight are, oldest first, B(i) R(i+D) B(i+1) ...
    # B(i+D-1) R(i+2D-1): vmcnt(2D-1) completes B(i), vmcnt(2D-2) R(i+D).
    a(".Lloop%=:")
    for u in range(R):
        s = u % D
        a("s_cmp_ge_u32 %[i], %[n]")
        a("s_cbranch_scc1 .Ldone%=")
        a(f"s_waitcnt vmcnt({2 * D - 1})")
        body(u)
        a(f"s_waitcnt vmcnt({2 * D - 2})")
        a(f"v_readfirstlane_b32 %[h{s}], v{(u + D) % R}")
        bload(f"h{s}", s)
        a(f"s_add_u32 %[t], %[i], {R}")
        a("s_min_u32 %[t], %[t], %[nm1]")
        a("s_lshl_b32 %[t], %[t], 6")
        a(f"buffer_load_dword v{u}, %[vro], %[rr], %[t] offen")
        a("s_add_u32 %[i], %[i], 1")
    a("s_branch .Lloop%=")
    a(".Ldone%=:")
    a("s_waitcnt vmcnt(0)")

    text = "".join(f'      "{x}\\n\\t"\n' for x in L)
    outs = ", ".join(f'"+{{v[{lo}:{hi}]}}"(acc.t[{q}])'
                     for q, (lo, hi) in enumerate(pl.tile_ranges()))
    clob = ", ".join(f'"v{r}"' for r in range(pl.nclob))
    hdecl = ", ".join(f"h{j}" for j in range(D))
    houts = ", ".join(f'[h{j}] "=&s"(h{j})' for j in range(D))
    return f"""// {mr} x {v} tile, {dt.upper()} B, {D} B rows in flight; tile at v{pl.base}
__device__ __forceinline__ void {pl.fn()}(Tile<{pl.nt}>& acc, uint32_t n,
                                       __amdgpu_buffer_rsrc_t rr, __amdgpu_buffer_rsrc_t rb,
                                       uint32_t ldbb, uint32_t km1, uint32_t vro, uint32_t vbo) {{
  uint32_t i, t, k, w, c, {hdecl};
  const uint32_t nm1 = n - 1;
  asm volatile(
{text}      : {outs}, [i] "=&s"(i), [t] "=&s"(t), [k] "=&s"(k), [w] "=&s"(w), [c] "=&s"(c),
        {houts}
      : [n] "s"(n), [nm1] "s"(nm1), [ldbb] "s"(ldbb), [km1] "s"(km1), [rr] "s"(rr), [rb] "s"(rb),
        [vro] "v"(vro), [vbo] "v"(vbo)
      : {clob}, "m0", "scc", "memory");
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
