"""Seeded synthetic inputs for Rosko SpMM workloads.

This module holds only random draws and data-layout helpers (masks, im2col).
It contains none of the method's arithmetic (no packing, no products), so it
can feed both the HIP path and the independent CPU oracle with the same
inputs.  Every generator takes an explicit seed and uses numpy's PCG64.

Workloads mirror the shapes the paper evaluates: unstructured weight sparsity
produced by magnitude pruning (Section 5.4) or uniform random sparsity
(Section 5.2), dense activations, and convolution-as-GEMM shapes (im2col).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# masks
# --------------------------------------------------------------------------
def bernoulli_mask(M: int, K: int, density: float, g: np.random.Generator) -> np.ndarray:
    """i.i.d. keep-mask: each entry kept with probability `density`."""
    return g.random((M, K)) < density


def magnitude_topk(W: np.ndarray, sparsity: float) -> np.ndarray:
    """Keep-mask of the k = round((1-s)*size) largest |W| entries.

    Ties in |W| are broken toward the lower row-major linear index (stable
    sort), so the mask is a deterministic function of W and s.
    """
    n = W.size
    k = int(round((1.0 - sparsity) * n))
    order = np.argsort(-np.abs(W).ravel(), kind="stable")
    keep = np.zeros(n, dtype=bool)
    keep[order[:k]] = True
    return keep.reshape(W.shape)


def row_clustered_mask(M: int, K: int, density: float, g: np.random.Generator) -> np.ndarray:
    """A fraction z ~ U(0, 0.5) of rows is all-zero, in contiguous runs; the
    remaining rows are Bernoulli with density d/(1-z) (capped at 1)."""
    z = g.uniform(0.0, 0.5)
    n_zero = int(round(z * M))
    zero_rows = np.zeros(M, dtype=bool)
    left = n_zero
    while left > 0:
        run = int(min(left, max(1, g.integers(1, max(2, M // 8) + 1))))
        start = int(g.integers(0, M))
        for i in range(run):
            r = (start + i) % M
            if not zero_rows[r]:
                zero_rows[r] = True
                left -= 1
                if left == 0:
                    break
    live = max(1, M - int(zero_rows.sum()))
    d_live = min(1.0, density * M / live)
    mask = g.random((M, K)) < d_live
    mask[zero_rows, :] = False
    return mask


def column_banded_mask(M: int, K: int, density: float, g: np.random.Generator) -> np.ndarray:
    """1-8 column bands with 10x the background keep-probability, scaled so
    that the expected density is `density`."""
    nb = int(g.integers(1, 9))
    weight = np.ones(K)
    for _ in range(nb):
        width = int(g.integers(max(1, K // 64), max(2, K // 8) + 1))
        start = int(g.integers(0, K))
        idx = (start + np.arange(width)) % K
        weight[idx] = 10.0
    p = density * K * weight / weight.sum()
    p = np.minimum(p, 1.0)
    return g.random((M, K)) < p[None, :]


def sparse_matrix(M: int, K: int, density: float, seed: int, kind: str = "iid") -> np.ndarray:
    """FP32 M x K matrix: N(0,1) values on a keep-mask of the given kind."""
    g = rng(seed)
    vals = g.standard_normal((M, K)).astype(np.float32)
    if kind == "iid":
        mask = bernoulli_mask(M, K, density, g)
    elif kind == "row_clustered":
        mask = row_clustered_mask(M, K, density, g)
    elif kind == "column_banded":
        mask = column_banded_mask(M, K, density, g)
    elif kind == "magnitude":
        mask = magnitude_topk(vals, 1.0 - density)
    else:
        raise ValueError(f"unknown mask kind {kind!r}")
    return np.where(mask, vals, np.float32(0.0)).astype(np.float32)


def dense_normal(R: int, C: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal((R, C)).astype(np.float32)


def im2col_3x3(X: np.ndarray) -> np.ndarray:
    """im2col of X (C, H, W) for a 3x3 kernel, stride 1, zero padding 1.

    Row index is c*9 + ky*3 + kx; column index is y*W + x.  Result is
    (9C) x (H*W) FP32, C-contiguous.
    """
    C, H, W = X.shape
    P = np.zeros((C, H + 2, W + 2), dtype=X.dtype)
    P[:, 1:H + 1, 1:W + 1] = X
    out = np.empty((C, 3, 3, H, W), dtype=X.dtype)
    for ky in range(3):
        for kx in range(3):
            out[:, ky, kx] = P[:, ky:ky + H, kx:kx + W]
    return np.ascontiguousarray(out.reshape(C * 9, H * W))


def bf16_representable(x: np.ndarray) -> np.ndarray:
    """Drop the low 16 bits of each FP32 value, so every value is exactly a
    BF16 number.  This draws BF16 activations; it is input generation and
    deliberately not the round-to-nearest encoding either implementation
    applies to the sparse operand."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    return b.view(np.float32).copy()


# --------------------------------------------------------------------------
# the evaluated workloads
# --------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    A: np.ndarray            # M x K FP32 (zeros are the pruned entries)
    B: np.ndarray            # K x N FP32 (or BF16-representable FP32)
    dC: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def plain_512(seed: int = 1) -> Problem:
    """A 512x512 with i.i.d. Bernoulli mask at 90% sparsity, N(0,1) values;
    B 512x512 N(0,1)."""
    g = rng(seed)
    vals = g.standard_normal((512, 512)).astype(np.float32)
    mask = bernoulli_mask(512, 512, 0.1, g)
    A = np.where(mask, vals, np.float32(0)).astype(np.float32)
    B = g.standard_normal((512, 512)).astype(np.float32)
    return Problem("plain-512-s90", A, B, meta={"sparsity": 0.9})


CNN_SPARSITIES = (0.70, 0.80, 0.90, 0.95, 0.99, 0.998)


def cnn_weights(sparsity: float, seed: int = 2, M: int = 256, K: int = 2304) -> np.ndarray:
    """Conv weights as a GEMM operand (256 out-channels x 256*3*3), N(0,1)
    draws pruned by magnitude to the given sparsity."""
    W = rng(seed).standard_normal((M, K)).astype(np.float32)
    keep = magnitude_topk(W, sparsity)
    return np.where(keep, W, np.float32(0)).astype(np.float32)


def cnn_activations(seed: int = 3, C: int = 256, H: int = 56, W: int = 56) -> np.ndarray:
    """im2col of ReLU(N(0,1)) activations of shape C x H x W (3x3, pad 1):
    a (9C) x (H*W) matrix, about half zeros, kept dense."""
    X = rng(seed).standard_normal((C, H, W)).astype(np.float32)
    X = np.maximum(X, np.float32(0))
    return im2col_3x3(X)


def cnn_layer(sparsity: float) -> Problem:
    A = cnn_weights(sparsity)
    B = cnn_activations()
    return Problem(f"cnn-256x2304x3136-s{sparsity:g}", A, B, meta={"sparsity": sparsity})


def precision_problem(sparsity: float, seed_a: int = 4, seed_b: int = 5,
                      M: int = 4096, K: int = 4096, N: int = 2048) -> Problem:
    """A M x K i.i.d. Bernoulli at the given sparsity, N(0,1) values (FP32
    source; the BF16/FP8 forms are encodings of it); B K x N N(0,1) truncated
    to BF16-representable values."""
    A = sparse_matrix(M, K, 1.0 - sparsity, seed_a, "iid")
    B = bf16_representable(dense_normal(K, N, seed_b))
    return Problem(f"prec-{M}x{K}x{N}-s{sparsity:g}", A, B, meta={"sparsity": sparsity})


def grad_problem(M: int = 1024, K: int = 4096, N: int = 1024, sparsity: float = 0.95,
                 seeds=(6, 7, 8)) -> Problem:
    A = sparse_matrix(M, K, 1.0 - sparsity, seeds[0], "iid")
    B = dense_normal(K, N, seeds[1])
    dC = dense_normal(M, N, seeds[2])
    return Problem(f"grad-{M}x{K}x{N}-s{sparsity:g}", A, B, dC, meta={"sparsity": sparsity})


MASK_KINDS = ("iid", "row_clustered", "column_banded")


def corpus_spec(i: int) -> dict:
    """Shape, sparsity and mask kind of corpus problem i (seed 10000+i):
    M, K log-uniform in [256, 8192], N log-uniform in [32, 4096], sparsity
    U(0.60, 0.998), mask kind cycling i.i.d. / row-clustered / column-banded."""
    g = rng(10000 + i)
    M = int(round(math.exp(g.uniform(math.log(256), math.log(8192)))))
    K = int(round(math.exp(g.uniform(math.log(256), math.log(8192)))))
    N = int(round(math.exp(g.uniform(math.log(32), math.log(4096)))))
    s = float(g.uniform(0.60, 0.998))
    kind = MASK_KINDS[i % 3]
    return {"i": i, "M": M, "K": K, "N": N, "sparsity": s, "kind": kind, "seed": 10000 + i}


def corpus_problem(i: int) -> Problem:
    sp = corpus_spec(i)
    A = sparse_matrix(sp["M"], sp["K"], 1.0 - sp["sparsity"], sp["seed"] + 1_000_000, sp["kind"])
    B = dense_normal(sp["K"], sp["N"], sp["seed"] + 2_000_000)
    return Problem(f"corpus-{i}", A, B, meta=sp)


def mlp_init_params(F: int, H: int, Cout: int, seed: int) -> dict:
    """He-uniform FP32 weights and zero biases for a
    Linear(F,H)-ReLU-Linear(H,H)-ReLU-Linear(H,Cout) network; W is [in, out]."""
    g = rng(seed)

    def lin(i, o):
        lim = math.sqrt(6.0 / i)
        return g.uniform(-lim, lim, size=(i, o)).astype(np.float32)

    return {"W1": lin(F, H), "b1": np.zeros(H, np.float32),
            "W2": lin(H, H), "b2": np.zeros(H, np.float32),
            "W3": lin(H, Cout), "b3": np.zeros(Cout, np.float32)}


def corpus_problem_device(i: int, device) -> tuple:
    """Corpus problem i generated on the GPU (torch's Philox generator seeded
    with the problem seed): A M x K FP32 with N(0,1) values on a keep-mask of
    the problem's kind, B K x N FP32 N(0,1).  The per-row and per-column
    structure of the row-clustered and column-banded masks (run positions,
    band positions) is drawn on the host with numpy exactly as in the host
    generators; the M x K and K x N random fields are drawn on the device.
    Used for the scheduler's timing corpus only (no oracle comparison)."""
    import torch
    sp = corpus_spec(i)
    M, K, N, d, kind = sp["M"], sp["K"], sp["N"], 1.0 - sp["sparsity"], sp["kind"]
    g = rng(sp["seed"] + 1_000_000)
    tg = torch.Generator(device=device)
    tg.manual_seed(sp["seed"])
    u = torch.rand((M, K), generator=tg, device=device)
    if kind == "iid":
        mask = u < d
    elif kind == "row_clustered":
        z = g.uniform(0.0, 0.5)
        n_zero = int(round(z * M))
        zero_rows = np.zeros(M, dtype=bool)
        left = n_zero
        while left > 0:
            run = int(min(left, max(1, g.integers(1, max(2, M // 8) + 1))))
            start = int(g.integers(0, M))
            for j in range(run):
                r = (start + j) % M
                if not zero_rows[r]:
                    zero_rows[r] = True
                    left -= 1
                    if left == 0:
                        break
        live = max(1, M - int(zero_rows.sum()))
        d_live = min(1.0, d * M / live)
        mask = (u < d_live) & torch.from_numpy(~zero_rows).to(device)[:, None]
    else:
        nb = int(g.integers(1, 9))
        weight = np.ones(K)
        for _ in range(nb):
            width = int(g.integers(max(1, K // 64), max(2, K // 8) + 1))
            start = int(g.integers(0, K))
            weight[(start + np.arange(width)) % K] = 10.0
        p = np.minimum(d * K * weight / weight.sum(), 1.0)
        mask = u < torch.from_numpy(p.astype(np.float32)).to(device)[None, :]
    del u
    vals = torch.randn((M, K), generator=tg, device=device)
    A = torch.where(mask, vals, torch.zeros((), device=device))
    del vals, mask
    B = torch.randn((K, N), generator=tg, device=device)
    return A, B, sp


SWEEP_N = (32, 64, 128, 256, 512, 1024, 2048, 3136)


def sweep_specs() -> list:
    """Matrices of the scheduler's measured sweep, each timed at every N in
    SWEEP_N: the shapes of the benchmark workloads (256 x 2304 convolution
    weights and their transpose, 1024 x 4096 and 4096 x 1024 from the
    gradient workload, 4096 x 4096 from the precision workload) plus 512 x 512
    and 2048 x 2048, over a range of sparsities and the three synthetic mask
    kinds (and magnitude pruning at the convolution shape).  Matrix j has seed
    20000 + j; every fourth matrix (j % 4 == 3) is held out of training."""
    wide = (0.6, 0.7, 0.8, 0.85, 0.9, 0.95, 0.97, 0.98, 0.99, 0.995, 0.998)
    narrow = (0.7, 0.85, 0.9, 0.95, 0.98, 0.995)
    groups = ((256, 2304, wide, MASK_KINDS + ("magnitude",)),
              (2304, 256, narrow, MASK_KINDS),
              (512, 512, narrow, MASK_KINDS),
              (1024, 4096, wide, MASK_KINDS),
              (4096, 1024, narrow, MASK_KINDS),
              (2048, 2048, narrow, MASK_KINDS),
              (4096, 4096, (0.6, 0.8, 0.9, 0.95, 0.98, 0.99, 0.998), ("iid",)),
              (4096, 4096, (0.9, 0.98), ("row_clustered", "column_banded")))
    out = []
    for M, K, sps, kinds in groups:
        for sp in sps:
            for kind in kinds:
                j = len(out)
                out.append({"j": j, "M": M, "K": K, "sparsity": sp, "kind": kind,
                            "seed": 20000 + j, "held_out": j % 4 == 3})
    return out


# --------------------------------------------------------------- graphs
@dataclass
class Graph:
    """A symmetric graph's GCN aggregation matrix in CSR form (FP32 values):
    row_ptr [n+1] int64, col_idx [nnz] int32 (ascending within a row),
    val [nnz] float32."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def sparsity(self) -> float:
        return 1.0 - self.nnz / float(self.n) ** 2


def power_law_graph(n: int, avg_degree: float, seed: int, exponent: float = 2.5,
                    cap_frac: float = 0.1) -> Graph:
    """Chung-Lu style random graph with a power-law expected degree sequence:
    node weights w_i from a Pareto law with tail exponent `exponent`
    (P(w > x) ~ x^(1 - exponent)) scaled to mean avg_degree and capped at
    cap_frac * n; each of the n * avg_degree / 2 edge draws picks both ends
    with probability proportional to w.  Both directions are stored,
    repeated draws and self-draws dropped, then every node gets its self
    loop and the GCN normalisation D^-1/2 (A + I) D^-1/2 (D the row counts
    including the loop).  Node ids carry no order (hubs land anywhere)."""
    g = rng(seed)
    shape = exponent - 1.0
    w = (1.0 - g.random(n)) ** (-1.0 / shape)
    for _ in range(8):                       # expected degrees, capped at cap_frac * n
        w = np.minimum(w / w.mean() * avg_degree, cap_frac * n)
    cw = np.cumsum(w)
    cw /= cw[-1]
    target = int(round(n * avg_degree / 2))
    keys = np.empty(0, np.int64)
    draws = target
    for _ in range(6):                       # top up what the de-duplication removed
        u = np.searchsorted(cw, g.random(draws), side="right").astype(np.int64)
        v = np.searchsorted(cw, g.random(draws), side="right").astype(np.int64)
        np.minimum(u, n - 1, out=u)
        np.minimum(v, n - 1, out=v)
        keep = u != v
        a, b = np.minimum(u[keep], v[keep]), np.maximum(u[keep], v[keep])
        keys = np.unique(np.concatenate([keys, a * n + b]))
        if keys.size >= target:
            break
        draws = int((target - keys.size) * 1.3) + 16
    if keys.size > target:
        keys = np.sort(g.choice(keys, target, replace=False))
    a, b = keys // n, keys % n
    loops = np.arange(n, dtype=np.int64)
    both = np.concatenate([a * n + b, b * n + a, loops * n + loops])
    both.sort()
    rows, cols = both // n, both % n
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    dinv = (1.0 / np.sqrt(counts.astype(np.float64)))
    val = (dinv[rows] * dinv[cols]).astype(np.float32)
    return Graph(n, row_ptr, cols.astype(np.int32), val)


# Graph shapes of the GCN aggregation experiment: the node counts and mean
# degrees of a social graph with 99.79% sparsity and of a protein association
# graph with 99.55% sparsity, and a 60000-node graph at 99.8% (7.3M entries);
# the feature lengths the experiment sweeps.
GCN_GRAPHS = {"social_233k": (232_965, 492.0, 11), "protein_133k": (132_534, 597.0, 12),
              "medium_60k": (60_000, 120.0, 911)}
GCN_FEATURES = (32, 64, 128, 256, 512)


def gcn_graph(name: str) -> Graph:
    n, deg, seed = GCN_GRAPHS[name]
    return power_law_graph(n, deg, seed)


def csr_to_dense(gr: Graph, perm: np.ndarray | None = None) -> np.ndarray:
    """Dense n x n FP32 array of the graph matrix (row i = CSR row perm[i]
    when a row order is given); small graphs only."""
    A = np.zeros((gr.n, gr.n), np.float32)
    rows = np.repeat(np.arange(gr.n), np.diff(gr.row_ptr))
    A[rows, gr.col_idx] = gr.val
    return A if perm is None else A[perm]
