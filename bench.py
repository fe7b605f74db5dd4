"""Benchmark of the Rosko hot path on one MI355X.

Workload: a pruned CNN layer as a GEMM -- weights A = 256 x 2304 (256
channels x 3x3 x 256), N(0,1) draws magnitude-pruned to 70/80/90/95/99/99.8%
sparsity, times the im2col activations B = 2304 x 3136 of a ReLU'd N(0,1)
256 x 56 x 56 input (about half zeros, kept dense), FP32.

One step packs each of the six weight matrices (count, scan, write) and
multiplies it with B (C = A B), i.e. one pass of the forward hot path over
the whole sparsity sweep.  value = sum over the sweep of 2*nnz*N divided by
the step time (effective GFLOP/s, FLOPs counted on stored nonzeros only).

Also reported: per-sparsity SpMM time and its fractions of the FP32
vector-ALU peak (2*nnz*N / time / 78.6 TFLOP/s) and of the HBM roofline
(algorithmic bytes / time / 8 TB/s), the dense FP32 GEMM time
(torch.matmul) for the speedup, cold-cache kernel times (a 512 MB buffer is
written between trials so the 256 MB Infinity Cache holds nothing of the
inputs), and the CPU oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 FMA on the vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
# Packed-FP32 forms (which would double it to the published 157.3 TFLOP/s)
# are switched off for all of the library's device code.
VALU_FP32_PEAK_TFS = 78.6
VALU_FP32_PUBLISHED_TFS = 157.3
SPMM_SOURCES = ("spmm_kernel.h", "spmm_loop.inc", "spmm.hip", "spmm_bf32.hip", "internal.h")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_spmm_rows_cnn_256x2304x3136_pmc.txt")


def _code_only(text):
    """C/C++ source without comments and with whitespace runs collapsed."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def spmm_sources_digest(read=None):
    """sha256 over the code of the SpMM kernels, comments and layout ignored
    (the counters below are only valid for the code they were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in SPMM_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, "paper_2307_03930_amd", "csrc", name)) as f:
                text = f.read()
        else:
            text = read(name)
        h.update(name.encode() + b"\0" + _code_only(text).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes of the six SpMM calls of one step, from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy of known size); None when the summary is missing or was taken on
    other kernel sources."""
    try:
        with open(PMC_SUMMARY) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    except OSError:
        return None
    if kv.get("sources_sha256", "").strip() != spmm_sources_digest():
        return None
    try:
        return int(kv["traffic_bytes_six_calls"].strip())
    except (KeyError, ValueError):
        return None


def alg_bytes(nnz, ncols, P, k_touched, N, M, s_val=4, s_b=4, s_c=4, beta=0):
    """Compulsory bytes of one SpMM: packed values + row bytes, column index
    and count per kept column, panel pointers, the touched rows of B, and C
    written (read too when beta = 1)."""
    return (nnz * (s_val + 1) + ncols * 8 + (P + 1) * 12 + k_touched * N * s_b
            + M * N * s_c * (1 + beta))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(As, B, mrs, budget_s: float = 20.0):
    """Time the CPU oracle (FP64 CSR loop, row-parallel) on a bounded sample
    of the same workload: all six matrices on every host thread (up to 16,
    the machine's CPU share), the 90% matrix on one thread, and the oracle's
    packer (Alg. 1) on each matrix at the panel height the GPU step uses."""
    import numpy as np
    import oracle as O
    O.build(force=False)
    threads = max(1, min(16, os.cpu_count() or 1))
    N = B.shape[1]
    nnzs = [int(np.count_nonzero(A.view(np.uint32) & np.uint32(0x7FFFFFFF))) for A in As]
    flops, t_total, reps = 0.0, 0.0, 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < budget_s / 2 or reps == 0:
        for A, nnz in zip(As, nnzs):
            t0 = time.perf_counter()
            O.spmm(A, B, threads=threads)
            t_total += time.perf_counter() - t0
            flops += 2.0 * nnz * N
        reps += 1
        if reps >= 3:
            break
    i90 = min(2, len(As) - 1)
    t0 = time.perf_counter()
    O.spmm(As[i90], B, threads=1)
    t1 = time.perf_counter() - t0
    pack_s = 0.0
    for A, mr in zip(As, mrs):
        t0 = time.perf_counter()
        O.pack(A, mr)
        pack_s += time.perf_counter() - t0
    return {"value": round(flops / t_total / 1e9, 3), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle", "cpu": _cpu_model(), "host_threads": os.cpu_count(),
            "single_thread_value": round(2.0 * nnzs[i90] * N / t1 / 1e9, 3),
            "single_thread_sample": "the 90% matrix once, one thread",
            "oracle_pack_ms_all_six": round(pack_s * 1e3, 2),
            "sample": f"{reps} pass(es) over all six sparsities of the 256x2304x3136 layer, "
                      f"FP64 CSR loop, {threads} threads"}


def _rel_err(x, ref, scale):
    """max |x - ref| / scale over the entries (3 significant digits)."""
    return float(f"{float(((x - ref).abs() / scale.clamp_min(1e-300)).max()):.3e}")


def _path_name(plan):
    return "dense-mfma" if plan is not None and plan.path == 1 else "sparse"


def _time_us(fn, reps, warm=3):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e3


def run_precision(args):
    """The precision forms: A 4096 x 4096 at 90% and 98% (i.i.d. mask, N(0,1)
    values) with values in FP32, BF16 or FP8 E4M3 + row scales, times B
    4096 x 2048 (BF16 for the BF16/FP8 forms, its FP32 copy for the FP32
    form); FP32 accumulation.  SpMM and packing timed separately."""
    import numpy as np
    import torch
    from paper_2307_03930_amd import ops, sched, synth
    torch.backends.cuda.matmul.allow_tf32 = False
    dev = torch.device("cuda:0")
    out = []
    dense_us = dense_bf16_us = None
    for sp in (0.90, 0.98):
        pr = synth.precision_problem(sp)
        A = torch.from_numpy(pr.A).to(dev)
        B32 = torch.from_numpy(pr.B).to(dev)
        B16 = B32.to(torch.bfloat16)
        M, K = pr.A.shape
        N = pr.B.shape[1]
        if dense_us is None:
            dense_us = _time_us(lambda: torch.matmul(A, B32), 10)
            A16 = A.to(torch.bfloat16).contiguous()
            dense_bf16_us = _time_us(lambda: torch.matmul(A16, B16), 10)
            del A16
        kt = int((pr.A != 0).any(axis=0).sum())
        # FP64 reference on the host (torch CPU): the exact product of the
        # FP32 source values and its |A||B| scale
        A64 = torch.from_numpy(pr.A).double()
        B64 = torch.from_numpy(pr.B).double()
        ref = A64 @ B64
        scale = A64.abs() @ B64.abs()
        del A64, B64
        for vals in ("f32", "bf16", "fp8"):
            mr, plan = sched.candidate(sched.choose(A, N, val_dtype=vals,
                                                    b_dtype="f32" if vals == "f32" else "bf16"))
            P = ops.pack(A, mr, vals)
            Bd = B32 if vals == "f32" else B16
            C = torch.empty((M, N), dtype=torch.float32, device=dev)
            ws = torch.empty(max(ops.spmm_workspace_size(P, N, plan), 1), dtype=torch.uint8,
                             device=dev)
            t = _time_us(lambda: ops.spmm(P, Bd, C, plan=plan, ws=ws), args.reps)
            e = _rel_err(C.cpu().double(), ref, scale)
            pws = torch.empty(max(ops.workspace_size(M, K, mr), 1), dtype=torch.uint8, device=dev)
            tp = _time_us(lambda: ops.pack_into(A, P, pws), args.reps)
            s_val = {"f32": 4, "bf16": 2, "fp8": 1}[vals]
            s_b = 4 if vals == "f32" else 2
            by = alg_bytes(P.nnz, P.ncols, (M + mr - 1) // mr, kt, N, M, s_val=s_val, s_b=s_b) + \
                (4 * M if vals == "fp8" else 0)
            fl = 2.0 * P.nnz * N
            out.append({"sparsity": sp, "values": vals, "B": "f32" if vals == "f32" else "bf16",
                        "mr": mr, "path": _path_name(plan), "nnz": P.nnz,
                        "spmm_us": round(t, 2), "pack_us": round(tp, 2),
                        "err_vs_fp64_fp32_source": e,
                        "gflops": round(fl / (t * 1e-6) / 1e9, 1),
                        "alu_frac": round(fl / (t * 1e-6) / 1e12 / VALU_FP32_PEAK_TFS, 3),
                        "hbm_frac": round(by / (t * 1e-6) / 1e9 / HBM_PEAK_GBS, 3),
                        "speedup_vs_dense_fp32": round(dense_us / t, 2),
                        "speedup_vs_dense_bf16": round(dense_bf16_us / t, 2)})
        del A, B32, B16, ref, scale
    print(json.dumps({"workload": "precision forms: A 4096x4096 at 90/98% (i.i.d.), values "
                                  "FP32/BF16/FP8+row scales, B 4096x2048, FP32 accumulate",
                      "unit": "us", "dense_fp32_gemm_us": round(dense_us, 2),
                      "dense_bf16_gemm_us": round(dense_bf16_us, 2),
                      "err": "max |C - C64| / (|A||B|), C64 the FP64 product of the FP32 source "
                             "values (torch CPU)", "data": "synthetic",
                      "forms": out}), flush=True)


def run_backward(args):
    """Forward and backward of C = A B: A 1024 x 4096 at 95% (i.i.d.), B
    4096 x 1024, dC 1024 x 1024, FP32.  dB = A^T dC through the packed
    transpose, dA = (dC B^T) on A's mask (SDDMM)."""
    import torch
    from paper_2307_03930_amd import ops, sched, synth
    torch.backends.cuda.matmul.allow_tf32 = False
    dev = torch.device("cuda:0")
    pr = synth.grad_problem()
    A = torch.from_numpy(pr.A).to(dev)
    B = torch.from_numpy(pr.B).to(dev)
    dC = torch.from_numpy(pr.dC).to(dev)
    M, K = pr.A.shape
    N = pr.B.shape[1]
    # One panel height serves the forward, the transposed pack and the
    # SDDMM: 8 rows (the SDDMM's LDS path covers panels of at most 8 rows),
    # the 8 x 4 register tile, the library's parallel shape.
    mr = 8
    P = ops.pack(A, mr, "f32")
    Pt = ops.pack_transpose(A, mr)
    plan = ops.make_plan(4)
    C = torch.empty((M, N), dtype=torch.float32, device=dev)
    ws = torch.empty(max(ops.spmm_workspace_size(P, N, plan), 1), dtype=torch.uint8, device=dev)
    n = P.nnz
    parts = {
        "pack_us": _time_us(lambda: ops.pack_into(A, P, P._ws), args.reps),
        "forward_spmm_us": _time_us(lambda: ops.spmm(P, B, C, plan=plan, ws=ws), args.reps),
        "dB_spmm_us": _time_us(lambda: ops.spmm_backward(P, Pt, B, dC, True, False), args.reps),
        "dA_sddmm_us": _time_us(lambda: ops.spmm_backward(P, Pt, B, dC, False, True), args.reps),
        "backward_us": _time_us(lambda: ops.spmm_backward(P, Pt, B, dC, True, True), args.reps),
    }
    dense_us = _time_us(lambda: torch.matmul(A, B), 10)
    fl = 2.0 * n * N
    res = {k: round(v, 2) for k, v in parts.items()}
    # errors against FP64 references on the host (torch CPU): dB = A^T dC,
    # dA = (dC B^T) on A's mask, scattered back to A's dense layout
    dA, dB = ops.spmm_backward(P, Pt, B, dC, True, True)
    dA_dense = torch.zeros((M, K), dtype=torch.float32, device=dev)
    ops.scatter_dense(P, dA, dA_dense)
    A64, B64, G64 = (torch.from_numpy(x).double() for x in (pr.A, pr.B, pr.dC))
    mask = A64 != 0
    rdB = A64.t() @ G64
    sdB = A64.abs().t() @ G64.abs()
    rdA = (G64 @ B64.t())[mask]
    sdA = (G64.abs() @ B64.abs().t())[mask]
    res["err_dB_vs_fp64"] = _rel_err(dB.cpu().double(), rdB, sdB)
    res["err_dA_vs_fp64"] = _rel_err(dA_dense.cpu().double()[mask], rdA, sdA)
    for k in ("forward_spmm_us", "dB_spmm_us", "dA_sddmm_us"):
        res[k.replace("_us", "_gflops")] = round(fl / (parts[k] * 1e-6) / 1e9, 1)
        res[k.replace("_us", "_alu_frac")] = round(fl / (parts[k] * 1e-6) / 1e12 /
                                                  VALU_FP32_PEAK_TFS, 3)
    print(json.dumps({"workload": "forward + backward: A 1024x4096 at 95% (i.i.d.), B 4096x1024, "
                                  "dC 1024x1024, FP32", "mr": mr, "nnz": n, "unit": "us",
                      "dense_fp32_gemm_us": round(dense_us, 2), "data": "synthetic", **res}),
          flush=True)


def run_training(args):
    """Pruned training with on-the-fly repacking (the training use of the
    method): one SGD step of the two-layer chain of the CNN layer -- a 3x3
    convolution 256 -> 256 channels (W1 256 x 2304) on the 56 x 56 im2col
    activations (2304 x 3136), ReLU, a 1x1 convolution 256 -> 256 (W2) --
    with both weights repacked every step, at several sparsities of both
    weights; beside it the same step with dense FP32 GEMMs (torch)."""
    import numpy as np
    import torch
    from paper_2307_03930_amd import autograd, synth, training
    torch.backends.cuda.matmul.allow_tf32 = False
    dev = torch.device("cuda:0")
    pr = synth.cnn_layer(0.9)
    X = torch.from_numpy(pr.B).to(dev)
    g = synth.rng(730)
    W1_0 = torch.from_numpy((g.standard_normal((256, 2304)) * 0.02).astype(np.float32)).to(dev)
    W2_0 = torch.from_numpy((g.standard_normal((256, 256)) * 0.06).astype(np.float32)).to(dev)
    T = torch.from_numpy(synth.dense_normal(256, 3136, 731)).to(dev)

    def dense_step(W1, W2):
        C2 = W2 @ torch.relu(W1 @ X)
        loss = ((C2 - T) ** 2).mean()
        loss.backward()
        with torch.no_grad():
            for W in (W1, W2):
                W -= 1e-3 * W.grad
                W.grad = None

    mr = args.mr if args.mr is not None else 8
    Wd1, Wd2 = W1_0.clone().requires_grad_(True), W2_0.clone().requires_grad_(True)
    dense_ms = _time_us(lambda: dense_step(Wd1, Wd2), 20, warm=20) / 1e3
    rows = []
    for s in (0.75, 0.80, 0.90, 0.95):
        W1, W2 = W1_0.clone(), W2_0.clone()
        training.magnitude_prune(W1, s)
        training.magnitude_prune(W2, s)
        chain = training.PrunedChain(W1, W2, mr)
        step_ms = _time_us(lambda: chain.step(X, T, 1e-3), 20, warm=20) / 1e3
        # the step's four packs (W1, W1^T, W2, W2^T) in its one batched call,
        # and as four separate calls
        pack_ms = _time_us(lambda: autograd.repack_weights([(chain.W1, chain.pw1),
                                                             (chain.W2, chain.pw2)]), 20) / 1e3
        sep_ms = _time_us(lambda: (chain.pw1.repack(chain.W1.detach()),
                                   chain.pw2.repack(chain.W2.detach())), 20) / 1e3
        chain.pw1.check()
        chain.pw2.check()
        rows.append({"sparsity": s, "step_ms": round(step_ms, 4), "repack_ms": round(pack_ms, 4),
                     "repack_separate_calls_ms": round(sep_ms, 4),
                     "speedup_vs_dense": round(dense_ms / step_ms, 2)})
    print(json.dumps({"workload": "pruned training step with repacking: W1 256x2304 (3x3 conv "
                                  "256->256) on im2col 2304x3136, ReLU, W2 256x256 (1x1 conv), "
                                  f"MSE loss, SGD; mr {mr}; FP32",
                      "unit": "ms", "dense_fp32_step_ms": round(dense_ms, 4),
                      "data": "synthetic", "per_sparsity": rows}), flush=True)


def run_gcn(args):
    """GCN aggregation (the graph workload): C = A X for the normalised
    adjacency A of a synthetic power-law graph (by default 60000 nodes, mean
    degree 120, 99.8% sparse), feature lengths 32..512, FP32.  A is packed
    from CSR on the GPU (mr 16) in the natural row order and in the
    inspector's balanced and degree orders; each SpMM is timed, and 150 sampled rows of
    each result are checked against an FP64 host reference.  The CPU
    baseline is the oracle's CSR product on a sample of rows."""
    import numpy as np
    import torch
    from paper_2307_03930_amd import ops, synth
    dev = torch.device("cuda:0")
    names = args.graphs.split(",") if args.graphs else ["medium_60k"]
    feats = synth.GCN_FEATURES
    mr = 16
    out = []
    for name in names:
        t0 = time.perf_counter()
        gr = synth.gcn_graph(name)
        print(f"# graph {name}: n={gr.n} nnz={gr.nnz} generated in "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        rp, ci, va = (torch.from_numpy(x).to(dev) for x in (gr.row_ptr, gr.col_idx, gr.val))
        rows = np.unique(synth.rng(77).integers(0, gr.n, 600))[::4]
        g = synth.rng(78)
        packs = {}
        for order in ("natural", "balanced", "degree"):
            t1 = time.perf_counter()
            perm = None if order == "natural" else ops.row_order(rp, mr, order)
            P = ops.pack_csr(rp, ci, va, gr.n, mr, "f32", perm)
            pack_ms = _time_us(lambda: ops.pack_csr_into(rp, ci, va, P, P._ws), 3,
                               warm=1) / 1e3
            order_ms = None
            if perm is not None:
                order_ms = _time_us(lambda: ops.row_order(rp, mr, order), 3, warm=1) / 1e3
            pan = np.add.reduceat(np.diff(gr.row_ptr)[perm.cpu().numpy()] if perm is not None
                                  else np.diff(gr.row_ptr), np.arange(0, gr.n, mr))
            packs[order] = (P, pack_ms, order_ms, float(pan.max() / pan.mean()))
            print(f"#   {order}: pack {pack_ms:.2f} ms, {P.nrec} records "
                  f"({time.perf_counter() - t1:.1f} s)", file=sys.stderr, flush=True)
        recs = []
        for N in feats:
            X = torch.from_numpy(g.standard_normal((gr.n, N), np.float32)).to(dev)
            C = torch.empty((gr.n, N), dtype=torch.float32, device=dev)
            Xh = X.cpu().double()
            refs = []
            for m in rows:
                b, en = int(gr.row_ptr[m]), int(gr.row_ptr[m + 1])
                a = torch.from_numpy(gr.val[b:en]).double()
                xs = Xh[torch.from_numpy(gr.col_idx[b:en].astype(np.int64))]
                refs.append((a @ xs, a.abs() @ xs.abs()))
            del Xh
            for order, (P, pack_ms, order_ms, spread) in packs.items():
                sw = torch.empty(max(ops.spmm_workspace_size(P, N), 1), dtype=torch.uint8,
                                 device=dev)
                t = _time_us(lambda: ops.spmm(P, X, C, ws=sw), 10, warm=2)
                Cs = C[torch.from_numpy(rows).to(dev)].cpu().double()
                e = max(float(((Cs[i] - r).abs() / sc.clamp_min(1e-300)).max())
                        for i, (r, sc) in enumerate(refs))
                recs.append({"order": order, "mr": mr, "N": N, "spmm_us": round(t, 1),
                             "gflops": round(2.0 * gr.nnz * N / (t * 1e-6) / 1e9, 1),
                             "err_sampled": float(f"{e:.3e}")})
                del sw
            print(f"#   N={N}: " + ", ".join(f"{r['order']} {r['spmm_us']} us"
                                             for r in recs[-len(packs):]),
                  file=sys.stderr, flush=True)
            del X, C
        res = {"graph": name, "n": gr.n, "nnz": gr.nnz, "sparsity": round(gr.sparsity, 5),
               "orders": {o: {"pack_ms": round(v[1], 2),
                              "row_order_ms": None if v[2] is None else round(v[2], 3),
                              "panel_entries_max_over_mean": round(v[3], 2),
                              "nrec": v[0].nrec}
                          for o, v in packs.items()},
               "spmm": recs}
        if not args.no_cpu_baseline:
            import oracle as O
            Xh = g.standard_normal((gr.n, 128), np.float32)
            sample = rows[:100]
            t1 = time.perf_counter()
            O.spmm_csr_rows(gr.row_ptr, gr.col_idx, gr.val, Xh, sample)
            dt = time.perf_counter() - t1
            nz = int(sum(gr.row_ptr[m + 1] - gr.row_ptr[m] for m in sample))
            res["cpu_baseline"] = {"value": round(2.0 * nz * 128 / dt / 1e9, 3),
                                   "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                                   "sample": "100 sampled rows at N=128, FP64 CSR rows"}
        out.append(res)
        del packs, rp, ci, va, gr
    print(json.dumps({"workload": "GCN aggregation C = A X, A the normalised adjacency of "
                                  "a synthetic power-law graph, FP32",
                      "unit": "us", "data": "synthetic", "graphs": out}), flush=True)


def run_conv(args):
    """Sparse direct convolution (no im2col) against the im2col route, for the
    pruned 3x3 layer of the CNN workload: 256 -> 256 channels on 56 x 56
    ReLU(N(0,1)) activations, weights pruned to 70..99.8%, FP32.  Direct: the
    shifted input copies plus the SpMM over the padded-pitch grid (the
    records remapped once per input size).  im2col route: the im2col matrix
    (torch unfold) plus the SpMM.  Same packed weight, panel height by the
    scheduler for the im2col product."""
    import numpy as np
    import torch
    import torch.nn.functional as F
    from paper_2307_03930_amd import ops, sched, synth
    dev = torch.device("cuda:0")
    X = torch.from_numpy(np.maximum(synth.rng(3).standard_normal((256, 56, 56)), 0)
                         .astype(np.float32)).to(dev)
    rows = []
    for sp in synth.CNN_SPARSITIES:
        A = torch.from_numpy(synth.cnn_weights(sp)).to(dev)
        mr, _ = sched.candidate(sched.choose(A, 3136))
        P = ops.pack(A, mr)
        layer = ops.ConvLayer(P, 256, 56, 56)
        Yq = torch.empty((256, 56 * layer.Wq), dtype=torch.float32, device=dev)
        C = torch.empty((256, 3136), dtype=torch.float32, device=dev)
        sw = torch.empty(max(ops.spmm_workspace_size(P, 3136), 1), dtype=torch.uint8,
                         device=dev)
        t_direct = _time_us(lambda: layer.run(X, Yq), args.reps)
        t_input = _time_us(lambda: ops.L.lib().rosko_conv_input(
            ops._ptr(X), 256, 56, 56, ops._ptr(layer.Bc), ops._stream_ptr()), args.reps)

        def im2col_route():
            B = F.unfold(X.unsqueeze(0), 3, padding=1)[0]
            ops.spmm(P, B, C, ws=sw)
        t_im2col = _time_us(im2col_route, args.reps)
        B = F.unfold(X.unsqueeze(0), 3, padding=1)[0].contiguous()
        t_spmm = _time_us(lambda: ops.spmm(P, B, C, ws=sw), args.reps)
        rows.append({"sparsity": sp, "mr": mr, "nnz": P.nnz,
                     "direct_us": round(t_direct, 2), "direct_input_copies_us": round(t_input, 2),
                     "im2col_route_us": round(t_im2col, 2), "spmm_on_im2col_us": round(t_spmm, 2),
                     "speedup_direct_vs_im2col_route": round(t_im2col / t_direct, 2)})
        del A, P, layer, Yq, C, sw, B
    print(json.dumps({"workload": "sparse direct 3x3 convolution 256->256 channels at 56x56 "
                                  "(stride 1, padding 1) vs im2col + SpMM, FP32",
                      "unit": "us", "data": "synthetic", "per_sparsity": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=50, help="kernel launches per timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip cold/dense timings")
    ap.add_argument("--cols-per-lane", type=int, default=None)
    ap.add_argument("--waves-per-tile", type=int, default=None)
    ap.add_argument("--k-split", type=int, default=None)
    ap.add_argument("--depth", type=int, default=None)
    ap.add_argument("--mr", type=int, default=None,
                    help="panel height for every matrix (default: the library's analytic "
                         "plan rule picks it per matrix)")
    ap.add_argument("--graphs", default=None, help="gcn workload: comma-separated graph names")
    ap.add_argument("--pack-mode", choices=("auto", "two_pass"), default="auto",
                    help="packing launches: one where the grid allows (auto) or the count "
                         "pass then the write (two_pass); the packed arrays are the same")
    ap.add_argument("--separate-packs", action="store_true",
                    help="cnn workload: re-pack each matrix in its own call right before its "
                         "SpMM, instead of one batched call (rosko_pack_batch) for all six")
    ap.add_argument("--workload", choices=("cnn", "precision", "backward", "training", "gcn",
                                           "conv"),
                    default="cnn",
                    help="cnn: the pruned-CNN sweep (the headline line); precision: the "
                         "BF16 / FP8 value forms at 4096x4096; backward: forward + backward "
                         "at 1024x4096")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    if args.pack_mode != "auto":
        from paper_2307_03930_amd import ops
        ops.set_pack_mode(args.pack_mode)

    if args.workload == "precision":
        return run_precision(args)
    if args.workload == "backward":
        return run_backward(args)
    if args.workload == "training":
        return run_training(args)
    if args.workload == "gcn":
        return run_gcn(args)
    if args.workload == "conv":
        return run_conv(args)

    import numpy as np
    import torch
    from paper_2307_03930_amd import ops, sched, synth

    torch.backends.cuda.matmul.allow_tf32 = False
    dev = torch.device("cuda:0")
    sparsities = list(synth.CNN_SPARSITIES)
    B_np = synth.cnn_activations()
    As_np = [synth.cnn_weights(s) for s in sparsities]
    M, K = As_np[0].shape
    N = B_np.shape[1]
    B = torch.from_numpy(B_np).to(dev)
    As = [torch.from_numpy(a).to(dev) for a in As_np]
    # per matrix, set up once outside the timed region: panel height and
    # register tile from the plan scheduler on the matrix's
    # statistics (unless given), the parallel shape from the library; buffers sized once
    # (the sizing query synchronises; the step does not)
    packs, wss, Cs, sws, plans, mrs = [], [], [], [], [], []
    for A in As:
        cols = args.cols_per_lane
        overrides = (cols, args.waves_per_tile, args.k_split, args.depth) != (None,) * 4
        if args.mr is None:
            mr, cand = sched.candidate(sched.choose(A, N))
            cols = cols or cand.cols_per_lane or 4
        else:
            mr, cand = args.mr, None
        if cand is not None and not overrides:
            plan = cand                      # the scheduler's candidate, sparse or dense
        else:
            plan = ops.make_plan(cols, args.waves_per_tile, args.k_split, args.depth)
        P = ops.pack(A, mr, "f32")
        packs.append(P)
        plans.append(plan)
        mrs.append(mr)
        wss.append(torch.empty(max(ops.workspace_size(M, K, mr), 1), dtype=torch.uint8,
                               device=dev))
        Cs.append(torch.empty((M, N), dtype=torch.float32, device=dev))
        sws.append(torch.empty(max(ops.spmm_workspace_size(P, N, plan), 1), dtype=torch.uint8,
                               device=dev))
    nnzs = [P.nnz for P in packs]
    ncolss = [P.ncols for P in packs]
    k_touched = [int((a != 0).any(axis=0).sum()) for a in As_np]

    batch = list(zip(As, packs, wss))

    def step():
        if args.separate_packs:
            for A, P, ws, C, sw, plan in zip(As, packs, wss, Cs, sws, plans):
                ops.pack_into(A, P, ws)
                ops.spmm(P, B, C, plan=plan, ws=sw)
        else:
            # the six re-packs in one call: matrices whose single pass has
            # the same kernel form share a grid (three launches here)
            ops.pack_batch_into(batch)
            for P, C, sw, plan in zip(packs, Cs, sws, plans):
                ops.spmm(P, B, C, plan=plan, ws=sw)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    flops_step = sum(2.0 * z * N for z in nnzs)
    value = flops_step / (ms_step * 1e-3) / 1e9

    # ---- per-sparsity SpMM kernel time (back-to-back launches, warm)
    per = []
    tot_bytes, tot_ms = 0.0, 0.0
    for s, P, C, sw, nnz, nc, kt, plan, mr in zip(sparsities, packs, Cs, sws, nnzs, ncolss,
                                                  k_touched, plans, mrs):
        P_panels = (M + mr - 1) // mr
        for _ in range(3):
            ops.spmm(P, B, C, plan=plan, ws=sw)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.reps):
            ops.spmm(P, B, C, plan=plan, ws=sw)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.reps
        by = alg_bytes(nnz, nc, P_panels, kt, N, M)
        A_s = As[sparsities.index(s)]
        ws_s = wss[sparsities.index(s)]
        pack_us = _time_us(lambda: ops.pack_into(A_s, P, ws_s), args.reps)
        tot_bytes += by
        tot_ms += ms
        per.append({"sparsity": s, "nnz": nnz, "mr": mr, "path": _path_name(plan),
                    "spmm_us": round(ms * 1e3, 2), "pack_us": round(pack_us, 2),
                    "gflops": round(2.0 * nnz * N / (ms * 1e-3) / 1e9, 1),
                    "alu_frac": round(2.0 * nnz * N / (ms * 1e-3) / 1e12 / VALU_FP32_PEAK_TFS, 3),
                    "alg_MB": round(by / 1e6, 2),
                    "hbm_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)})

    extras = {}
    if not args.no_extras:
        # dense FP32 GEMM at the same shape (hipBLASLt through torch), warm
        Ad = As[2]
        for _ in range(3):
            torch.matmul(Ad, B)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            torch.matmul(Ad, B)
        b.record()
        torch.cuda.synchronize()
        dense_us = a.elapsed_time(b) / 20 * 1e3
        extras["dense_fp32_gemm_us"] = round(dense_us, 2)
        for rec in per:
            rec["speedup_vs_dense"] = round(dense_us / rec["spmm_us"], 2)
        # a plain 256 MB device copy: the known-size reference that hardware
        # traffic counters (FETCH_SIZE / WRITE_SIZE) are scaled by
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        extras["copy_reference_bytes"] = int(src.numel() * 4)
        del src, dst
        # per-call distributions over 50 trials (median, p10, p90): warm calls
        # back to back, each between its own pair of events; cold calls after
        # overwriting 512 MB (twice the last-level cache) and synchronising
        def dist(ts):
            return {"median": round(float(np.median(ts)), 2),
                    "p10": round(float(np.percentile(ts, 10)), 2),
                    "p90": round(float(np.percentile(ts, 90)), 2)}
        trials = 50
        flush = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device=dev)
        for rec, P, C, sw, plan in zip(per, packs, Cs, sws, plans):
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(trials)]
            for a, b in ev:
                a.record()
                ops.spmm(P, B, C, plan=plan, ws=sw)
                b.record()
            torch.cuda.synchronize()
            rec["spmm_warm_us"] = dist([a.elapsed_time(b) * 1e3 for a, b in ev])
            ts = []
            for _ in range(trials):
                flush.fill_(1.0)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                ops.spmm(P, B, C, plan=plan, ws=sw)
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b) * 1e3)
            rec["spmm_cold_us"] = dist(ts)
            rec["spmm_cold_us_median"] = rec["spmm_cold_us"]["median"]
        del flush

    hbm_achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    tot_flops = sum(2.0 * z * N for z in nnzs)
    alu_achieved = tot_flops / (tot_ms * 1e-3) / 1e12
    out = {
        "metric": "SpMM effective GFLOP/s (2*nnz*N/t)",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "pruned-CNN conv-as-GEMM FP32: A 256x2304 magnitude-pruned at "
                               "70/80/90/95/99/99.8%, B 2304x3136 im2col(ReLU(N(0,1))); "
                               "step = pack + SpMM for all six",
                   "pack_calls": "per matrix" if args.separate_packs else "one batched call",
                   "M": M, "K": K, "N": N,
                   "mr": args.mr if args.mr is not None else
                   f"per matrix, {sched.chooser_name()} scheduler",
                   "pack_mode": args.pack_mode,
                   "parallelism": "single-gpu"},
        # the SpMM call (k_spmm_rows, then k_reduce_splits when K is split),
        # one launch per sparsity, timed back to back with events on the
        # stream it runs on; FLOPs on stored nonzeros only
        "roofline": {"bound": "alu", "achieved": round(alu_achieved, 3),
                     "peak": VALU_FP32_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": round(alu_achieved / VALU_FP32_PEAK_TFS, 4),
                     "traffic": measured_traffic(),
                     "frac_vs_published_peak": round(alu_achieved / VALU_FP32_PUBLISHED_TFS, 4),
                     "kernel": "k_spmm_rows + k_reduce_splits (rosko_spmm)",
                     "launches": len(per), "alg_bytes": int(tot_bytes),
                     "hbm_achieved_GBs": round(hbm_achieved, 1),
                     "hbm_frac": round(hbm_achieved / HBM_PEAK_GBS, 4)},
        "per_sparsity": per,
    }
    out.update(extras)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(As_np, B_np, mrs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
