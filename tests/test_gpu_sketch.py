"""GPU parity of the hash and the sketch application against the oracle.

Bar: hash buckets and signs bit-exact; S A bit-exact (the kernels sum each
sketch row in the sequential order of the definition, so float64 results are
identical, not merely close); reduced-precision outputs equal the oracle's
single rounding of the float64 sum; two runs bitwise equal."""
import numpy as np
import pytest

import workloads as W
from oracle import sketch as OS

pytestmark = pytest.mark.gpu


def dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    if t.dtype == torch.bfloat16:
        t = t.double()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,m,s,problem,seed,it", [
    (1000, 500, 1, 0, 7, 0), (4097, 4096, 4, 0, 2 ** 63 + 5, 9),
    (333, 48, 3, 2, 1, 2 ** 40), (1, 1, 1, 0, 0, 0), (70000, 8192, 1, 5, 123, 4)])
def test_hash_bit_exact(gpu_lib, n, m, s, problem, seed, it):
    P = gpu_lib
    kind = "sjlt" if s > 1 else "countsketch"
    b, sg = P.sketch_hash(n, P.SketchSpec(m, s, kind, seed, it), problem=problem)
    rb, rs = OS.sketch_hash(seed, it, n, m, s, problem)
    assert np.array_equal(host(b), rb)
    assert np.array_equal(host(sg), rs)


CASES = [  # n, d, m, s
    (5000, 50, 500, 1),      # odd width, one load per lane
    (3000, 256, 64, 1),      # two chunks of 128 columns
    (2048, 512, 256, 4),     # SJLT
    (777, 130, 1024, 1),     # n < m: empty buckets, ragged column tail
    (1, 7, 16, 1),           # single row
    (900, 1, 32, 2),         # single column, SJLT s=2 (scale after the sum)
    (4000, 1024, 128, 1),    # widest dense path
    (1500, 600, 96, 3),      # 600 columns (paired loads), s = 3
    (40000, 8, 16384, 1),    # largest sketch: a 64 KiB LDS histogram per sort tile
    (300, 5, 1, 1),          # one sketch row: every row in one bucket
    (70000, 16, 4096, 4),    # many sort tiles, SJLT over 4 blocks
    (600, 20, 16, 16),       # SJLT with one bucket per block: every row in every sketch row
    # two sketch rows per wavefront, long lists paired with short ones:
    (6000, 96, 4098, 2),     # odd block length (2049): one wavefront spans both blocks
    (3000, 200, 2048, 1),    # about one row per sketch row: many equal list lengths
    (20000, 72, 16384, 1),   # block longer than the pairing takes: natural order
]


@pytest.mark.parametrize("n,d,m,s", CASES)
def test_dense_sketch_bit_exact(gpu_lib, n, d, m, s):
    P = gpu_lib
    g = np.random.default_rng(n * 7 + d)
    A = g.standard_normal((n, d))
    kind = "sjlt" if s > 1 else "countsketch"
    spec = P.SketchSpec(m, s, kind, seed=11, iter=3)
    SA = P.sketch_apply(P.Matrix(dense=dev(A)), spec)
    ref = OS.sketch_apply_dense(A, 11, 3, m, s)
    assert np.array_equal(host(SA), ref)


def test_dense_sketch_reduced_outputs_and_f32_input(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(1)
    A = g.standard_normal((3000, 200))
    spec = P.SketchSpec(128, 1, seed=4, iter=1)
    M = P.Matrix(dense=dev(A))
    for dt in ("float32", "bfloat16"):
        out = host(P.sketch_apply(M, spec, out_dtype=dt))
        assert np.array_equal(out.astype(np.float64),
                              OS.sketch_apply_dense(A, 4, 1, 128, 1, out_dtype=dt).astype(np.float64))
    A32 = A.astype(np.float32)
    out = host(P.sketch_apply(P.Matrix(dense=dev(A32)), spec))
    assert np.array_equal(out, OS.sketch_apply_dense(A32, 4, 1, 128, 1))


@pytest.mark.parametrize("n,d", [(3000, 512), (2000, 1000), (5000, 132), (700, 130)])
def test_dense_sketch_f32_rows_bit_exact(gpu_lib, n, d):
    """float32 rows: quads of floats per lane when the width allows, pairs or
    single elements otherwise; the sum is still formed in float64."""
    P = gpu_lib
    g = np.random.default_rng(d)
    A32 = g.standard_normal((n, d)).astype(np.float32)
    spec = P.SketchSpec(256, 1, seed=12, iter=2)
    out = host(P.sketch_apply(P.Matrix(dense=dev(A32)), spec))
    assert np.array_equal(out, OS.sketch_apply_dense(A32, 12, 2, 256, 1))


def test_dense_sketch_strided_rows(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(2)
    big = g.standard_normal((800, 80))
    A = dev(big)[:, :70]          # leading dimension 80, width 70
    spec = P.SketchSpec(40, 1, seed=9)
    out = host(P.sketch_apply(P.Matrix(dense=A), spec))
    assert np.array_equal(out, OS.sketch_apply_dense(big[:, :70], 9, 0, 40, 1))


def test_sketch_deterministic(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(3)
    M = P.Matrix(dense=dev(g.standard_normal((20000, 256))))
    spec = P.SketchSpec(1024, 4, "sjlt", seed=5)
    a = P.sketch_apply(M, spec)
    b = P.sketch_apply(M, spec)
    assert bool((a == b).all())


def test_empty_matrix_gives_zero_sketch(gpu_lib):
    import torch
    P = gpu_lib
    A = torch.empty(0, 16, dtype=torch.float64, device="cuda")
    out = P.sketch_apply(P.Matrix(dense=A), P.SketchSpec(8))
    assert bool((out == 0).all())


@pytest.mark.parametrize("n,d,density,m,s", [(3000, 40, 0.05, 64, 1), (20000, 300, 0.01, 512, 4),
                                             (500, 1024, 0.002, 16, 1), (100, 5, 0.0, 8, 1),
                                             (800, 30, 0.2, 8, 8), (300, 1024, 0.2, 32, 2),
                                             (40000, 64, 0.05, 16384, 1)])
def test_csr_sketch_bit_exact(gpu_lib, n, d, density, m, s):
    """Bit-exact against the oracle's sequential definition, with rows of
    ~200 nonzeros (several 64-entry batches per row) and the largest number
    of sketch rows (the sort's two LDS histograms at their largest)."""
    P = gpu_lib
    import torch
    wl = W.ridge_csr(rows=n, d=d, density=density, m=m)
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=n, d=d)
    kind = "sjlt" if s > 1 else "countsketch"
    out = host(P.sketch_apply(M, P.SketchSpec(m, s, kind, seed=6, iter=2)))
    ref = OS.sketch_apply_csr(wl.indptr, wl.indices, wl.data, n, d, 6, 2, m, s)
    assert np.array_equal(out, ref)


def csr_rows(wl, r0, r1):
    """Rows r0 .. r1 of a CSR workload as a CSR matrix of their own."""
    lo, hi = int(wl.indptr[r0]), int(wl.indptr[r1])
    return wl.indptr[r0:r1 + 1] - lo, wl.indices[lo:hi], wl.data[lo:hi], r1 - r0


@pytest.mark.parametrize("s", [1, 4])
def test_csr_ragged_batch_sketch(gpu_lib, s):
    """A ragged batch of CSR problems (rows of one CSR matrix split by
    row_offsets, an empty problem among them): each problem's sketch
    bit-exact against the oracle's on its own rows, with its own hash
    stream."""
    P = gpu_lib
    wl = W.ridge_csr(rows=9000, d=200, density=0.02, m=512)
    offs = np.array([0, 3000, 3000, 3001, 9000])
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d, row_offsets=offs)
    kind = "sjlt" if s > 1 else "countsketch"
    m = 512
    out = host(P.sketch_apply(M, P.SketchSpec(m, s, kind, seed=6, iter=2)))
    for p in range(len(offs) - 1):
        ip, ix, dv, n_p = csr_rows(wl, offs[p], offs[p + 1])
        ref = OS.sketch_apply_csr(ip, ix, dv, n_p, wl.d, 6, 2, m, s, problem=p)
        assert np.array_equal(out[p * m:(p + 1) * m], ref), p


def test_csr_hot_column_ordering(gpu_lib):
    """Every row hits column 0: each wavefront batch holds 64 equal columns."""
    P = gpu_lib
    n, d, m = 5000, 12, 8
    g = np.random.default_rng(4)
    rows = []
    for i in range(n):
        cols = np.unique(np.concatenate([[0], g.choice(d, size=g.integers(0, 4))]))
        rows.append(cols)
    indptr = np.zeros(n + 1, dtype=np.int32)
    indptr[1:] = np.cumsum([len(c) for c in rows])
    indices = np.concatenate(rows).astype(np.int32)
    data = g.standard_normal(len(indices))
    M = P.Matrix(row_ptr=dev(indptr), col_idx=dev(indices), values=dev(data), n=n, d=d)
    out = host(P.sketch_apply(M, P.SketchSpec(m, seed=1)))
    assert np.array_equal(out, OS.sketch_apply_csr(indptr, indices, data, n, d, 1, 0, m, 1))


def test_ragged_batch_sketch(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(5)
    sizes = [300, 1, 0, 2500, 64]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    A = g.standard_normal((offs[-1], 64))
    m = 40
    out = host(P.sketch_apply(P.Matrix(dense=dev(A), row_offsets=offs), P.SketchSpec(m, seed=8)))
    for p in range(len(sizes)):
        ref = OS.sketch_apply_dense(A[offs[p]:offs[p + 1]], 8, 0, m, 1, problem=p)
        assert np.array_equal(out[p * m:(p + 1) * m], ref), p


@pytest.mark.parametrize("sizes,s", [([3000, 0, 1, 2500], 1), ([0, 0, 0], 1),
                                     ([3000, 0, 1, 2500], 4), ([2500, 700], 2)])
def test_ragged_batch_two_rows_per_wave(gpu_lib, sizes, s):
    """Batches wide enough (batch * m >= 2048, 64 < d <= 768) for the paired
    two-rows-per-wavefront gather, with empty problems, a batch of empty
    problems only (every list empty), and SJLT blocks (pairs formed within
    each block; m = 1026 at s = 2 gives blocks of odd length)."""
    P = gpu_lib
    g = np.random.default_rng(len(sizes) + s)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    d = 80
    m = 1026 if s == 2 else 1024
    kind = "sjlt" if s > 1 else "countsketch"
    A = g.standard_normal((offs[-1], d))
    M = P.Matrix(dense=dev(A.reshape(-1, d)), row_offsets=offs)
    out = host(P.sketch_apply(M, P.SketchSpec(m, s, kind, seed=12, iter=2)))
    for p in range(len(sizes)):
        ref = OS.sketch_apply_dense(A[offs[p]:offs[p + 1]], 12, 2, m, s, problem=p)
        assert np.array_equal(out[p * m:(p + 1) * m], ref), p


@pytest.mark.parametrize("s", [1, 4, 16])
def test_sketch_adjoint(gpu_lib, s):
    P = gpu_lib
    g = np.random.default_rng(6)
    n, d, m = 3000, 64, 256
    G = g.standard_normal((m, d))
    kind = "sjlt" if s > 1 else "countsketch"
    out = host(P.sketch_adjoint(dev(G), n, P.SketchSpec(m, s, kind, seed=3, iter=1)))
    assert np.array_equal(out, OS.sketch_adjoint(G, n, 3, 1, m, s))


def test_sketch_adjoint_ragged(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(7)
    sizes = [100, 0, 350]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    m, d = 32, 16
    G = g.standard_normal((len(sizes) * m, d))
    out = host(P.sketch_adjoint(dev(G), int(offs[-1]), P.SketchSpec(m, seed=2), row_offsets=offs))
    for p in range(len(sizes)):
        ref = OS.sketch_adjoint(G[p * m:(p + 1) * m], sizes[p], 2, 0, m, 1, problem=p)
        assert np.array_equal(out[offs[p]:offs[p + 1]], ref)


def test_sketch_adjoint_many_problems(gpu_lib):
    """More problems than one launch takes (70 > 64), empty and one-row
    problems, 64-row groups that straddle problems, d = 100 (a ragged column
    tail) and an SJLT with s = 4: bit-exact per problem."""
    P = gpu_lib
    g = np.random.default_rng(71)
    sizes = g.integers(0, 200, 70)
    sizes[[3, 40, 64]] = 0
    sizes[[5, 65]] = 1
    offs = np.concatenate([[0], np.cumsum(sizes)])
    m, d, s = 48, 100, 4
    G = g.standard_normal((len(sizes) * m, d))
    out = host(P.sketch_adjoint(dev(G), int(offs[-1]), P.SketchSpec(m, s, "sjlt", seed=12, iter=3),
                                row_offsets=offs))
    for p in range(len(sizes)):
        ref = OS.sketch_adjoint(G[p * m:(p + 1) * m], int(sizes[p]), 12, 3, m, s, problem=p)
        assert np.array_equal(out[offs[p]:offs[p + 1]], ref), p
