"""Oracle: the sparse embeddings of Sec. 2 (CountSketch and SJLT), their hash,
their application to dense and CSR data, and their adjoint.

Hash (the paper leaves the family open; this library's choice):
  key      = (seed, iteration)                     two uint64 words
  counter  = (i, k // 2, p, 0)                     row i (0-based, local to
                                                   problem p), block pair k//2
  words    = Philox4x64-10(counter, key) = (w0, w1, w2, w3)
  block k uses wb = w[2 (k mod 2)] for its row and ws = w[2 (k mod 2) + 1]
  for its sign:
      local row  = floor(wb * m_blk / 2^64)        (m_blk = m / s)
      sign       = -1 if the top bit of ws is set, else +1
      sketch row = k * m_blk + local row

CountSketch is s = 1: column i of S has a single +-1 at row h(i) (Sec. 2).
SJLT stacks s independent CountSketches of m/s rows each (Sec. 2), and its
entries carry the 1/sqrt(s) normalisation that makes E[S^T S] = I
(App. A.1.1, the remark before Def. A.3, and Lemma A.7).

Sketch application (Sec. 2, "Time Complexity of sketching methods": one pass
over the nonzeros, each nonzero A_ij adds +-A_ij into bucket (h(i), j)):
  SA[r, :] = c_s * sum over rows i hashed to sketch row r, taken in
             ascending i and added one at a time from +0.0, of sign(i) A[i, :]
  with c_s = 1/sqrt(s) applied once to the finished sum (c_1 = 1 is not
  applied). Accumulation is float64 whatever the input type; an output in
  float32 or bfloat16 is the float64 sum rounded to nearest-even once.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import mulhilo64, philox4x64


# --------------------------------------------------------------------------
# hash
# --------------------------------------------------------------------------
def sketch_hash(seed, iteration, n, m, s=1, problem=0):
    """Bucket (sketch row) and sign of every (row, block) pair.

    Returns bucket int64 (n, s) with values in [0, m) and sign int8 (n, s)."""
    if s < 1 or m % s:
        raise ValueError("SJLT needs s >= 1 dividing m")
    m_blk = m // s
    rows = np.arange(n, dtype=np.uint64)
    bucket = np.empty((n, s), dtype=np.int64)
    sign = np.empty((n, s), dtype=np.int8)
    cache = {}
    for k in range(s):
        q = k // 2
        if q not in cache:
            cache[q] = philox4x64(rows, q, problem, 0, seed, iteration)
        w = cache[q]
        wb, ws = w[2 * (k % 2)], w[2 * (k % 2) + 1]
        hi, _ = mulhilo64(wb, np.uint64(m_blk))
        bucket[:, k] = k * m_blk + hi.astype(np.int64)
        sign[:, k] = np.where((ws >> np.uint64(63)) != 0, -1, 1)
    return bucket, sign


def block_scale(s):
    """Entry magnitude of an SJLT with s blocks (1 for CountSketch)."""
    return 1.0 / math.sqrt(s)


def dense_sketch_matrix(seed, iteration, n, m, s=1, problem=0):
    """Explicit m x n matrix S (tiny sizes only; brute-force checks)."""
    bucket, sign = sketch_hash(seed, iteration, n, m, s, problem)
    S = np.zeros((m, n))
    c = block_scale(s)
    for k in range(s):
        S[bucket[:, k], np.arange(n)] = sign[:, k] * c
    return S


# --------------------------------------------------------------------------
# rounding helpers for reduced-precision outputs
# --------------------------------------------------------------------------
def round_to_bf16(x):
    """Round float64 values to the nearest bfloat16 (ties to even) in a single
    rounding, returned as float64 values. Normal-range inputs only."""
    x = np.asarray(x, dtype=np.float64)
    bits = x.view(np.uint64)
    drop = np.uint64(52 - 7)              # bfloat16 keeps 7 fraction bits
    lsb = (bits >> drop) & np.uint64(1)
    bias = (np.uint64(1) << (drop - np.uint64(1))) - np.uint64(1) + lsb
    with np.errstate(over="ignore"):
        r = (bits + bias) & ~((np.uint64(1) << drop) - np.uint64(1))
    out = r.view(np.float64).copy()
    finite = np.isfinite(x)
    out[~finite] = x[~finite]
    return out


def round_output(x, dtype):
    if dtype in ("float64", np.float64):
        return np.asarray(x, dtype=np.float64)
    if dtype in ("float32", np.float32):
        return np.asarray(x, dtype=np.float64).astype(np.float32)
    if dtype == "bfloat16":
        return round_to_bf16(x)
    raise ValueError(dtype)


# --------------------------------------------------------------------------
# application
# --------------------------------------------------------------------------
def _ranks_within_groups(keys):
    """For keys already sorted so equal keys are adjacent, the 0-based position
    of each element inside its run of equal keys."""
    n = len(keys)
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    start = np.ones(n, dtype=bool)
    start[1:] = keys[1:] != keys[:-1]
    run_start = np.maximum.accumulate(np.where(start, np.arange(n), 0))
    return np.arange(n) - run_start


def sketch_apply_dense(A, seed, iteration, m, s=1, problem=0,
                       out_dtype="float64"):
    """SA for dense A (n x d), summed sequentially per sketch row in ascending
    input-row order. Each round adds the r-th row of every bucket, so no bucket
    receives two rows in one vectorised update and the order is exact."""
    A = np.asarray(A)
    n, d = A.shape
    bucket, sign = sketch_hash(seed, iteration, n, m, s, problem)
    rows = np.tile(np.arange(n)[:, None], (1, s)).ravel()
    bk = bucket.ravel()
    sg = sign.ravel().astype(np.float64)
    order = np.lexsort((rows, bk))        # by bucket, then ascending row
    rows, bk, sg = rows[order], bk[order], sg[order]
    rank = _ranks_within_groups(bk)
    SA = np.zeros((m, d), dtype=np.float64)
    Af = A.astype(np.float64, copy=False)
    for r in range(int(rank.max()) + 1 if len(rank) else 0):
        sel = rank == r
        b_sel = bk[sel]
        SA[b_sel] = SA[b_sel] + sg[sel][:, None] * Af[rows[sel]]
    if s > 1:
        SA = SA * block_scale(s)
    return round_output(SA, out_dtype)


def sketch_apply_csr(indptr, indices, data, n, d, seed, iteration, m, s=1,
                     problem=0, out_dtype="float64"):
    """SA (dense m x d) for CSR A with canonical rows (sorted, unique columns),
    summed per (sketch row, column) in ascending input-row order."""
    indptr = np.asarray(indptr, dtype=np.int64)
    cols = np.asarray(indices, dtype=np.int64)
    vals = np.asarray(data, dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(indptr))
    bucket, sign = sketch_hash(seed, iteration, n, m, s, problem)
    SA = np.zeros((m, d), dtype=np.float64)
    nz_b = np.concatenate([bucket[rows, k] for k in range(s)]) if len(rows) else np.zeros(0, np.int64)
    nz_c = np.tile(cols, s)
    nz_r = np.tile(rows, s)
    nz_v = np.concatenate([sign[rows, k] * vals for k in range(s)]) if len(rows) else np.zeros(0)
    order = np.lexsort((nz_r, nz_c, nz_b))      # by (bucket, column), then row
    nz_b, nz_c, nz_r, nz_v = nz_b[order], nz_c[order], nz_r[order], nz_v[order]
    rank = _ranks_within_groups(nz_b * d + nz_c)
    for r in range(int(rank.max()) + 1 if len(rank) else 0):
        sel = rank == r
        SA[nz_b[sel], nz_c[sel]] = SA[nz_b[sel], nz_c[sel]] + nz_v[sel]
    if s > 1:
        SA = SA * block_scale(s)
    return round_output(SA, out_dtype)


def sketch_adjoint(G, n, seed, iteration, m, s=1, problem=0):
    """S^T G for G (m x d): row i of the result is the sum over blocks k, in
    ascending k from +0.0, of sign(i,k) * (c_s * G[bucket(i,k), :])."""
    G = np.asarray(G, dtype=np.float64)
    bucket, sign = sketch_hash(seed, iteration, n, m, s, problem)
    c = block_scale(s)
    out = np.zeros((n, G.shape[1]))
    for k in range(s):
        term = G[bucket[:, k]]
        if s > 1:
            term = term * c
        out = out + sign[:, k].astype(np.float64)[:, None] * term
    return out
