"""Seeded synthetic inputs for the constrained least-squares problems of
Eq.(1), shaped like the five workloads this library is measured on.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws data; it holds none of the sketching or solver arithmetic.

Data model: the Gaussian design of Sec. 1 (b = A x* + w, w_i ~ N(0, sigma^2)).
Constraint sets: C = R^d, the l1 ball or the l2 ball (Sec. 1, Eq.(1)).

Workloads (full sizes; every generator takes a row count override so tests can
run the same recipe at small n):

  ols_dense      20000 x 50, A ~ N(0,1), CountSketch m=500, 10 steps, C = R^d
  lasso_dense    2^20 x 256, rows ~ N(0, Sigma), Sigma_ij = 0.5^|i-j| (exact
                 AR(1) recursion per row), x* with round(0.1 d) nonzeros,
                 ||x||_1 <= 0.9 ||x*||_1, CountSketch or SJLT(s=4), m=4096
  ridge_csr      2^22 x 1024 CSR at density 1e-3, rows uniform, columns from a
                 Zipf(1.1) pmf truncated to d columns (column 0 hottest),
                 values N(0,1), duplicates summed, ||x||_2 <= ||x*||_2, m=8192
  precision      2^22 x 512, A = G diag(sigma) V, G ~ N(0,1) drawn in fp32,
                 sigma log-spaced 1 .. 1e-5, V Haar orthogonal, A stored fp64,
                 CountSketch m=4096, C = R^d
  batch_ragged   64 problems, n_i uniform in [16384, 131072], d = 64,
                 m = 10 d, 20 steps, target y ~ N(0,1) for L = ||x - y||^2
  table1_like    CSR stand-ins with the shape and density of the datasets of
                 App. B, Table 1 (default: W8A, 49749 x 300 at 4%): rows
                 uniform, columns from a truncated Zipf(1.1) pmf, values 1.0
                 for the binary-feature W*A sets and N(0,1) otherwise; used
                 for the sketch-error sweep of App. B, Fig. 2

Two backends draw the same recipe: "numpy" (CPU float64, used at test sizes)
and "torch" (any torch device, used at full size on the GPU). They use
different random streams, so their values differ; a test always hands the
same arrays to both sides of a comparison.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 20191031

FULL_ROWS = {
    "ols_dense": 20000,
    "lasso_dense": 1 << 20,
    "ridge_csr": 1 << 22,
    "precision": 1 << 22,
}


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    d: int
    b: object                      # (n,) float64
    x_star: object                 # (d,) or (B, d)
    constraint: str                # "none" | "l1" | "l2" | "l1_penalty"
    radius: float                  # ball radius, or lambda for "l1_penalty"
    sketch_kind: str               # "countsketch" | "sjlt"
    m: int
    s: int
    iters: int
    sketch_seed: int
    A: object = None               # dense (n, d), row-major
    indptr: object = None          # CSR row pointers (n+1,), int32
    indices: object = None         # CSR column indices (nnz,), int32
    data: object = None            # CSR values (nnz,), float64
    row_offsets: Optional[np.ndarray] = None   # ragged batch (B+1,), int64
    y: object = None               # batch targets (B, d)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def is_csr(self) -> bool:
        return self.indptr is not None

    @property
    def batch(self) -> int:
        return 1 if self.row_offsets is None else len(self.row_offsets) - 1


def _np_rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# ols_dense: plain Gaussian design
# --------------------------------------------------------------------------
def ols_dense(rows=None, d=50, m=500, iters=10, seed=BASE_SEED + 0,
              backend="numpy", device=None, dtype="float64"):
    n = FULL_ROWS["ols_dense"] if rows is None else int(rows)
    if backend == "numpy":
        g = _np_rng(seed)
        A = g.standard_normal((n, d))
        x_star = g.standard_normal(d)
        b = A @ x_star + 0.1 * g.standard_normal(n)
        if dtype == "float32":
            A = A.astype(np.float32)
    else:
        import torch
        gen = torch.Generator(device=device).manual_seed(seed)
        A = torch.randn(n, d, generator=gen, device=device, dtype=torch.float64)
        x_star = torch.randn(d, generator=gen, device=device, dtype=torch.float64)
        b = A @ x_star + 0.1 * torch.randn(n, generator=gen, device=device,
                                           dtype=torch.float64)
        if dtype == "float32":
            A = A.float()
    return Workload("ols_dense", n, d, b, x_star, "none", 0.0, "countsketch",
                    m, 1, iters, seed + 1000, A=A)


# --------------------------------------------------------------------------
# lasso_dense: AR(1) rows, sparse ground truth, active l1 ball
# --------------------------------------------------------------------------
def lasso_dense(rows=None, d=256, m=4096, sketch="countsketch", s=None,
                iters=20, seed=BASE_SEED + 1, backend="numpy", device=None, penalty=None):
    """LASSO data. By default the constrained form with the ball ||x||_1 <=
    0.9 ||x*||_1; with `penalty` = lambda, the penalised form
    1/2 ||Ax - b||^2 + lambda ||x||_1 of the paper's experiments (lambda = 5)."""
    n = FULL_ROWS["lasso_dense"] if rows is None else int(rows)
    if s is None:
        s = 4 if sketch == "sjlt" else 1
    k_nz = max(1, int(round(0.1 * d)))
    rho, c = 0.5, math.sqrt(1.0 - 0.25)
    if backend == "numpy":
        g = _np_rng(seed)
        Z = g.standard_normal((n, d))
        A = np.empty((n, d))
        A[:, 0] = Z[:, 0]
        for j in range(1, d):
            A[:, j] = rho * A[:, j - 1] + c * Z[:, j]
        del Z
        support = g.choice(d, size=k_nz, replace=False)
        x_star = np.zeros(d)
        x_star[support] = g.standard_normal(k_nz)
        b = A @ x_star + 0.1 * g.standard_normal(n)
        tau = 0.9 * float(np.abs(x_star).sum())
    else:
        import torch
        gen = torch.Generator(device=device).manual_seed(seed)
        A = torch.empty(n, d, device=device, dtype=torch.float64)
        prev = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
        A[:, 0] = prev
        for j in range(1, d):
            z = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
            prev = rho * prev + c * z
            A[:, j] = prev
        perm = torch.randperm(d, generator=gen, device=device)[:k_nz]
        x_star = torch.zeros(d, device=device, dtype=torch.float64)
        x_star[perm] = torch.randn(k_nz, generator=gen, device=device,
                                   dtype=torch.float64)
        b = A @ x_star + 0.1 * torch.randn(n, generator=gen, device=device,
                                           dtype=torch.float64)
        tau = 0.9 * float(x_star.abs().sum())
    if penalty is not None:
        return Workload("lasso_dense", n, d, b, x_star, "l1_penalty", float(penalty), sketch,
                        m, s, iters, seed + 1000, A=A)
    return Workload("lasso_dense", n, d, b, x_star, "l1", tau, sketch, m, s,
                    iters, seed + 1000, A=A)


# --------------------------------------------------------------------------
# ridge_csr: sparse rows, Zipf(1.1) column popularity, active/inactive l2 ball
# --------------------------------------------------------------------------
def zipf_pmf(d, a=1.1):
    """Zipf(a) pmf truncated to the ranks 1..d (rank k maps to column k-1)."""
    k = np.arange(1, d + 1, dtype=np.float64)
    p = k ** (-a)
    return p / p.sum()


def ridge_csr(rows=None, d=1024, density=1e-3, m=8192, iters=15,
              seed=BASE_SEED + 2, radius_factor=1.0):
    """CSR problem. Always drawn with numpy (the CSR build is host work);
    the caller moves the arrays to the device."""
    n = FULL_ROWS["ridge_csr"] if rows is None else int(rows)
    g = _np_rng(seed)
    nnz_target = int(round(density * n * d))
    r = g.integers(0, n, size=nnz_target, dtype=np.int64)
    cols = g.choice(d, size=nnz_target, p=zipf_pmf(d)).astype(np.int64)
    vals = g.standard_normal(nnz_target)
    # canonical CSR: sort by (row, col) and sum duplicates
    key = r * d + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(start) else vals[:0]
    rows_u = uniq // d
    cols_u = (uniq % d).astype(np.int32)
    counts = np.bincount(rows_u, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    x_star = g.standard_normal(d)
    noise = g.standard_normal(n)
    # b = A x* + 0.01 w, evaluated row by row from the CSR arrays
    prod = np.zeros(n)
    np.add.at(prod, rows_u, summed * x_star[cols_u])
    b = prod + 0.01 * noise
    radius = radius_factor * float(np.linalg.norm(x_star))
    assert indptr[-1] < 2 ** 31
    return Workload("ridge_csr", n, d, b, x_star, "l2", radius, "countsketch",
                    m, 1, iters, seed + 1000,
                    indptr=indptr.astype(np.int32), indices=cols_u,
                    data=summed.astype(np.float64),
                    meta={"nnz": int(indptr[-1])})


# --------------------------------------------------------------------------
# precision: A = G diag(sigma) V, condition number 1e5
# --------------------------------------------------------------------------
def precision_sigma(d, kappa=1e5):
    k = np.arange(d, dtype=np.float64)
    return 10.0 ** (-math.log10(kappa) * k / (d - 1)) if d > 1 else np.ones(1)


def haar_orthogonal_np(d, g):
    Q, R = np.linalg.qr(g.standard_normal((d, d)))
    return Q * np.sign(np.diag(R))


def precision(rows=None, d=512, m=4096, iters=60, kappa=1e5,
              seed=BASE_SEED + 3, backend="numpy", device=None,
              keep_factors=False, chunk_rows=1 << 18):
    n = FULL_ROWS["precision"] if rows is None else int(rows)
    sigma = precision_sigma(d, kappa)
    if backend == "numpy":
        g = _np_rng(seed)
        G = g.standard_normal((n, d), dtype=np.float32)
        V = haar_orthogonal_np(d, g)
        A = (G.astype(np.float64) * sigma) @ V
        x_star = g.standard_normal(d)
        b = A @ x_star + 0.1 * g.standard_normal(n)
    else:
        import torch
        gen = torch.Generator(device=device).manual_seed(seed)
        Q, R = torch.linalg.qr(torch.randn(d, d, generator=gen, device=device,
                                           dtype=torch.float64))
        V = Q * torch.sign(torch.diagonal(R))
        sig = torch.tensor(sigma, device=device, dtype=torch.float64)
        A = torch.empty(n, d, device=device, dtype=torch.float64)
        G = torch.empty(n, d, device=device, dtype=torch.float32) if keep_factors else None
        for r0 in range(0, n, chunk_rows):
            r1 = min(n, r0 + chunk_rows)
            Gc = torch.randn(r1 - r0, d, generator=gen, device=device,
                             dtype=torch.float32)
            if G is not None:
                G[r0:r1] = Gc
            A[r0:r1] = (Gc.double() * sig) @ V
        x_star = torch.randn(d, generator=gen, device=device, dtype=torch.float64)
        b = A @ x_star + 0.1 * torch.randn(n, generator=gen, device=device,
                                           dtype=torch.float64)
    meta = {"sigma": sigma, "V": V, "kappa": kappa}
    if backend == "numpy" and keep_factors:
        meta["G"] = G
    elif backend != "numpy" and keep_factors:
        meta["G"] = G
    return Workload("precision", n, d, b, x_star, "none", 0.0, "countsketch",
                    m, 1, iters, seed + 1000, A=A, meta=meta)


# --------------------------------------------------------------------------
# batch_ragged: many small OLS problems of uneven height, one target each
# --------------------------------------------------------------------------
def batch_ragged(num=64, n_lo=16384, n_hi=131072, d=64, m=None, iters=20,
                 seed=BASE_SEED + 4, backend="numpy", device=None,
                 dtype="float64"):
    m = 10 * d if m is None else m
    g = _np_rng(seed)
    sizes = g.integers(n_lo, n_hi + 1, size=num).astype(np.int64)
    row_offsets = np.zeros(num + 1, dtype=np.int64)
    np.cumsum(sizes, out=row_offsets[1:])
    N = int(row_offsets[-1])
    if backend == "numpy":
        A = g.standard_normal((N, d))
        x_star = g.standard_normal((num, d))
        b = np.empty(N)
        for p in range(num):
            r0, r1 = row_offsets[p], row_offsets[p + 1]
            b[r0:r1] = A[r0:r1] @ x_star[p] + 0.1 * g.standard_normal(r1 - r0)
        y = g.standard_normal((num, d))
        if dtype == "float32":
            A = A.astype(np.float32)
    else:
        import torch
        gen = torch.Generator(device=device).manual_seed(seed)
        A = torch.randn(N, d, generator=gen, device=device, dtype=torch.float64)
        x_star = torch.randn(num, d, generator=gen, device=device,
                             dtype=torch.float64)
        b = torch.empty(N, device=device, dtype=torch.float64)
        for p in range(num):
            r0, r1 = int(row_offsets[p]), int(row_offsets[p + 1])
            b[r0:r1] = A[r0:r1] @ x_star[p] + 0.1 * torch.randn(
                r1 - r0, generator=gen, device=device, dtype=torch.float64)
        y = torch.randn(num, d, generator=gen, device=device, dtype=torch.float64)
        if dtype == "float32":
            A = A.float()
    return Workload("batch_ragged", N, d, b, x_star, "none", 0.0,
                    "countsketch", m, 1, iters, seed + 1000, A=A,
                    row_offsets=row_offsets, y=y)


# --------------------------------------------------------------------------
# table1_like: sparse stand-ins with the shapes and densities of Table 1
# --------------------------------------------------------------------------
TABLE1 = {  # name: (n, d, density), App. B, Table 1
    "abtaha": (37932, 330, 0.01),
    "specular": (477976, 50, 0.01),
    "w4a": (7366, 300, 0.04),
    "w6a": (17188, 300, 0.04),
    "w8a": (49749, 300, 0.04),
    "yearpredictionmsd": (515344, 90, 1.0),
}


def table1_like(name="w8a", rows=None, seed=BASE_SEED + 5, values=None):
    """CSR matrix with Table 1's shape and density for `name`. Nonzero
    positions: rows uniform, columns from the Zipf(1.1) pmf truncated to d;
    repeated positions are drawn again until the target count of distinct
    positions is reached. Values: 1.0 for the W*A sets (binary features),
    N(0,1) otherwise (or as `values` says: "binary" | "gaussian").
    b = A x* + 0.1 w with x* ~ N(0,1); the LASSO weight of Sec. 3 (5.0) is
    carried as the radius."""
    n0, d, density = TABLE1[name.lower()]
    n = n0 if rows is None else int(rows)
    if values is None:
        values = "binary" if name.lower().startswith("w") else "gaussian"
    g = _np_rng(seed)
    target = int(round(density * n * d))
    pmf = zipf_pmf(d)
    keys = np.empty(0, dtype=np.int64)
    while len(keys) < target:
        need = target - len(keys)
        r = g.integers(0, n, size=need + need // 8 + 16, dtype=np.int64)
        c = g.choice(d, size=len(r), p=pmf).astype(np.int64)
        keys = np.unique(np.concatenate([keys, r * d + c]))
    keys = np.sort(g.permutation(keys)[:target])   # an unbiased subset, sorted
    rows_u = keys // d
    cols_u = (keys % d).astype(np.int32)
    if values == "binary":
        data = np.ones(target)
    else:
        data = g.standard_normal(target)
    counts = np.bincount(rows_u, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    x_star = g.standard_normal(d)
    prod = np.zeros(n)
    np.add.at(prod, rows_u, data * x_star[cols_u])
    b = prod + 0.1 * g.standard_normal(n)
    return Workload(name.lower() + "_like", n, d, b, x_star, "l1_penalty", 5.0,
                    "countsketch", 10 * d, 1, 20, seed + 1000,
                    indptr=indptr.astype(np.int32), indices=cols_u, data=data,
                    meta={"nnz": target, "density": density})


def csr_to_dense(indptr, indices, data, n, d):
    """Dense copy of a CSR matrix (test helper; tiny sizes only)."""
    out = np.zeros((n, d))
    indptr = np.asarray(indptr, dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(indptr))
    out[rows, np.asarray(indices)] = np.asarray(data)
    return out
