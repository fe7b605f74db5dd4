"""FP64 oracle for the scheduler's packing statistics (16 features of a
dense M x K matrix A multiplied by a K x N matrix).

TEST INFRASTRUCTURE ONLY.  Plain numpy on the definitions below; shares no
code with the GPU kernels.  "Nonzero" is the packing test of Alg. 1
(Sec. 4.1): a value is kept when its bits, sign masked off, are not all zero
(so -0.0 is dropped and NaN / subnormals are kept).  Panels of r rows are the
row blocks [p*r, min(M, p*r + r)), as packing cuts them; a kept panel column
is a (panel, k) pair with at least one kept value (a column Alg. 1 emits).

  f0  log2 M            f1  log2 K             f2  log2 N
  f3  d = nnz / (M K)   f4  log10(d + 1e-6)
  f5  coefficient of variation (population std / mean) of the row counts
  f6  fraction of rows with no kept value
  f7  coefficient of variation of the column counts
  f8  fraction of columns with no kept value
  f9  nnz / (kept panel columns at r = 32)          (values per column, 32-row panels)
  f10 (kept panel columns at r = 32) / (ceil(M/32) K)
  f11 nnz / (kept panel columns at r = 8)
  f12 coefficient of variation of the 32-row panel counts
  f13 max / mean of the 32-row panel counts
  f14 log2(1 + nnz N)   f15 log2(M N)
A ratio whose denominator is zero is 0.
"""
from __future__ import annotations

import numpy as np

NFEAT = 16


def kept_mask(A: np.ndarray) -> np.ndarray:
    bits = np.ascontiguousarray(A, dtype=np.float32).view(np.uint32)
    return (bits & np.uint32(0x7FFFFFFF)) != 0


def _cv(x: np.ndarray) -> float:
    x = np.asarray(x, np.float64)
    if x.size == 0 or x.mean() == 0:
        return 0.0
    return float(x.std() / x.mean())


def _ratio(a: float, b: float) -> float:
    return float(a) / float(b) if b else 0.0


def kept_panel_columns(mask: np.ndarray, r: int) -> int:
    M, K = mask.shape
    total = 0
    for p0 in range(0, M, r):
        total += int(mask[p0:p0 + r].any(axis=0).sum())
    return total


def features(A: np.ndarray, N: int) -> np.ndarray:
    mask = kept_mask(A)
    M, K = mask.shape
    nnz = int(mask.sum())
    rows = mask.sum(axis=1)
    cols = mask.sum(axis=0)
    P32 = (M + 31) // 32
    panels = np.array([mask[p * 32:(p + 1) * 32].sum() for p in range(P32)], np.float64)
    c32 = kept_panel_columns(mask, 32)
    c8 = kept_panel_columns(mask, 8)
    d = nnz / (M * K) if M * K else 0.0
    f = np.zeros(NFEAT, np.float64)
    f[0], f[1], f[2] = np.log2(M), np.log2(K), np.log2(N)
    f[3] = d
    f[4] = np.log10(d + 1e-6)
    f[5] = _cv(rows)
    f[6] = float((rows == 0).mean()) if M else 0.0
    f[7] = _cv(cols)
    f[8] = float((cols == 0).mean()) if K else 0.0
    f[9] = _ratio(nnz, c32)
    f[10] = _ratio(c32, P32 * K)
    f[11] = _ratio(nnz, c8)
    f[12] = _cv(panels)
    f[13] = _ratio(panels.max() if panels.size else 0.0, panels.mean() if panels.size else 0.0)
    f[14] = np.log2(1.0 + nnz * float(N))
    f[15] = np.log2(float(M) * float(N))
    return f
