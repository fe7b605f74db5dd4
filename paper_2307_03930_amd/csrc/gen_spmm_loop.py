"""Writes spmm_loop.inc: the record loop of the row-skipping SpMM (Alg. 2)
as one inline-asm block per (register tile, B dtype).

Why generated: the loop keeps 4 columns' B rows and 8 column records in
flight with vector loads and waits for each with an exact vmcnt.  Written as
C++ the compiler's wait-count analysis falls back to vmcnt(0) at the head of
the unrolled loop, draining the pipeline every 8 columns; a single asm block
owns every load it issues and waits for all of them before it ends, so no
load is ever in flight outside the block.

Register use inside the block (listed as clobbers / pinned operands):
  v0..v7     column records, slot u holds record i with i % 8 == u
             (lane l holds dword l & 15 of the 16-dword record)
  v8..v23    B row units, slot s = i % 4 (V elements per lane)
  v24..v27   BF16 units widened to FP32
  tile       v40.. (128-register tiles) or v32.. (smaller), column j of
             row r at base + j*MR + r
Per column: the header (k << 8 | count) is read with v_readfirstlane,
min(k, K-1) * ldb * elem becomes the SGPR offset of a buffer load of the B row; the
values are broadcast from the record register with DPP row_newbcast into
v_fmac_f32 whose accumulator is addressed relative to the row byte
(s_set_gpr_idx_on, SRC2 and DST).

Run `python gen_spmm_loop.py` after changing it; a CPU test checks that the
committed spmm_loop.inc matches.
"""
import os

TILES = [(8, 4), (16, 4), (32, 2), (32, 4), (64, 2), (128, 1)]
DTYPES = ["f32", "bf16"]
D = 4          # B rows in flight
R = 2 * D      # record slots


def tile_base(mr, v):
    return 40 if mr * v == 128 else 32


def tile_ranges(mr, v):
    base = tile_base(mr, v)
    nt = mr * v // 32
    return [(base + 32 * q, base + 32 * q + 31) for q in range(nt)]


def b_slot_regs(dt, v, s):
    """(load destination text, per-element FP32 register names, conversion asm)."""
    if dt == "f32":
        lo = 8 + v * s
        dst = f"v[{lo}:{lo + v - 1}]" if v > 1 else f"v{lo}"
        return dst, [f"v{lo + j}" for j in range(v)], []
    # bf16: V/2 dwords (or one ushort) per unit, widened into v24..
    if v == 4:
        lo = 8 + 2 * s
        conv = [f"v_lshlrev_b32 v24, 16, v{lo}", f"v_and_b32 v25, 0xffff0000, v{lo}",
                f"v_lshlrev_b32 v26, 16, v{lo + 1}", f"v_and_b32 v27, 0xffff0000, v{lo + 1}"]
        return f"v[{lo}:{lo + 1}]", ["v24", "v25", "v26", "v27"], conv
    lo = 8 + s
    if v == 2:
        conv = [f"v_lshlrev_b32 v24, 16, v{lo}", f"v_and_b32 v25, 0xffff0000, v{lo}"]
        return f"v{lo}", ["v24", "v25"], conv
    return f"v{lo}", ["v24"], [f"v_lshlrev_b32 v24, 16, v{lo}"]


def b_load_op(dt, v):
    nbytes = v * (4 if dt == "f32" else 2)
    return {16: "buffer_load_dwordx4", 8: "buffer_load_dwordx2", 4: "buffer_load_dword",
            2: "buffer_load_ushort"}[nbytes]


def gen_variant(mr, v, dt):
    base = tile_base(mr, v)
    mask = "0x%08x" % ((mr - 1) * 0x01010101)
    cols = [base + j * mr for j in range(v)]
    L = []

    def a(x):
        L.append(x)

    def rload_const(j):
        a(f"s_min_u32 %[t], {j}, %[nm1]")
        a("s_lshl_b32 %[t], %[t], 6")
        a(f"buffer_load_dword v{j}, %[vro], %[rr], %[t] offen")

    def bload(h, s):
        dst, _, _ = b_slot_regs(dt, v, s)
        a(f"s_lshr_b32 %[k], %[{h}], 8")
        a("s_min_u32 %[k], %[k], %[km1]")        # keeps every B access in bounds
        a("s_mul_i32 %[k], %[k], %[ldbb]")
        a(f"{b_load_op(dt, v)} {dst}, %[vbo], %[rb], %[k] offen")

    def body(u):
        s = u % D
        _, bregs, conv = b_slot_regs(dt, v, s)
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

    # ---- prologue: records 0..3, then for each: header, B row, record j+4
    a("s_mov_b32 %[i], 0")
    for j in range(D):
        rload_const(j)
    for j in range(D):
        a(f"s_waitcnt vmcnt({D - 1 + j})")
        a(f"v_readfirstlane_b32 %[h{j}], v{j}")
        bload(f"h{j}", j)
        rload_const(D + j)
    # ---- steady state, unrolled over the 8 record slots
    a(".Lloop%=:")
    for u in range(R):
        s = u % D
        a("s_cmp_ge_u32 %[i], %[n]")
        a("s_cbranch_scc1 .Ldone%=")
        a(f"s_waitcnt vmcnt({2 * D - 1})")       # B row of column i
        body(u)
        a(f"s_waitcnt vmcnt({2 * D - 2})")       # record of column i + 4
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
    nt = mr * v // 32
    outs = ", ".join(f'"+{{v[{lo}:{hi}]}}"(acc.t[{q}])'
                     for q, (lo, hi) in enumerate(tile_ranges(mr, v)))
    clob = ", ".join(f'"v{r}"' for r in range(28))
    fn = f"rk_loop_{mr}x{v}_{dt}"
    return f"""// {mr} x {v} tile, {dt.upper()} B
__device__ __forceinline__ void {fn}(Tile<{nt}>& acc, uint32_t n, __amdgpu_buffer_rsrc_t rr,
                                       __amdgpu_buffer_rsrc_t rb, uint32_t ldbb, uint32_t km1,
                                       uint32_t vro, uint32_t vbo) {{
  uint32_t i, t, k, w, c, h0, h1, h2, h3;
  const uint32_t nm1 = n - 1;
  asm volatile(
{text}      : {outs}, [i] "=&s"(i), [t] "=&s"(t), [k] "=&s"(k), [w] "=&s"(w), [c] "=&s"(c),
        [h0] "=&s"(h0), [h1] "=&s"(h1), [h2] "=&s"(h2), [h3] "=&s"(h3)
      : [n] "s"(n), [nm1] "s"(nm1), [ldbb] "s"(ldbb), [km1] "s"(km1), [rr] "s"(rr), [rb] "s"(rb),
        [vro] "v"(vro), [vbo] "v"(vbo)
      : {clob}, "m0", "scc", "memory");
}}
"""


def generate():
    out = ["// Generated by gen_spmm_loop.py -- do not edit.\n"
           "// Record loops of the row-skipping SpMM, one per (tile, B dtype); see the\n"
           "// generator for the register plan and the pipeline.\n"
           "#pragma once\n"]
    for mr, v in TILES:
        for dt in DTYPES:
            out.append(gen_variant(mr, v, dt))
    out.append("""template <int MR, int V, int TB> struct RkLoop;
""")
    for mr, v in TILES:
        for dt, tb in (("f32", "ROSKO_F32"), ("bf16", "ROSKO_BF16")):
            nt = mr * v // 32
            out.append(f"""template <> struct RkLoop<{mr}, {v}, {tb}> {{
  static __device__ __forceinline__ void run(Tile<{nt}>& acc, uint32_t n,
                                             __amdgpu_buffer_rsrc_t rr, __amdgpu_buffer_rsrc_t rb,
                                             uint32_t ldbb, uint32_t km1, uint32_t vro,
                                             uint32_t vbo) {{
    rk_loop_{mr}x{v}_{dt}(acc, n, rr, rb, ldbb, km1, vro, vbo);
  }}
}};
""")
    return "\n".join(out)


PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spmm_loop.inc")

if __name__ == "__main__":
    with open(PATH, "w") as f:
        f.write(generate())
    print("wrote", PATH)
