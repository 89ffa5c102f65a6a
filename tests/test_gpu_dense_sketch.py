"""GPU parity of the dense sketches of Sec. 2 (SRHT and Gaussian) against
the oracle, and of IHS run with them.

SRHT: the library's transform takes the butterflies of the radix-2
recursion in the recursion's order, so S A is bitwise the oracle's (float64,
and the float32 / bfloat16 outputs rounded once from it).
Gaussian: the entries of G come from log, sqrt, cos and sin, which the two
sides evaluate with different libraries (each within a few units in the
last place), and the product is summed in another order, so S A is compared
componentwise against |dSA| <= c_m (gamma_n |G||A| + 16 u R|A|) + u |SA| for
each side (R: the Box-Muller radius bounding each |G| entry; 16 u bounds the
error of one generated entry relative to R: a few ulps from log, sqrt and
the product, and 2 pi u2 rounded before cos and sin on the oracle's side)."""
import math

import numpy as np
import pytest

import rounding_budget as RB
import workloads as W
from oracle import dense_sketch as DS
from oracle import ihs as O
from oracle import sketch as OS

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.double().cpu().numpy()


def gauss_bound(A, seed, it, m):
    n = A.shape[0]
    G, R = DS.gaussian_matrix(seed, it, m, n, with_radius=True)
    aa = np.abs(A)
    gamma = n * U / (1 - n * U)
    ref = (G @ A) * (1.0 / math.sqrt(m))
    return 2 * ((gamma * (np.abs(G) @ aa) + 16 * U * (R @ aa)) / math.sqrt(m)
                + U * np.abs(ref))


@pytest.mark.parametrize("n,d,m", [(1000, 33, 200), (1024, 64, 512), (1, 5, 3), (3, 17, 9),
                                   (5000, 300, 600), (1 << 17, 16, 1000),
                                   ((1 << 20) + 3, 8, 64)])
def test_srht_bit_exact(gpu_lib, n, d, m):
    P = gpu_lib
    g = np.random.default_rng(n + d)
    A = g.standard_normal((n, d))
    spec = P.SketchSpec(m, kind="srht", seed=31, iter=n % 7)
    out = host(P.sketch_apply(P.Matrix(dense=dev(A)), spec))
    ref = DS.sketch_apply_srht(A, 31, n % 7, m)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("dt", ["float32", "bfloat16"])
def test_srht_float32_data_and_rounded_outputs(gpu_lib, dt):
    import torch
    P = gpu_lib
    g = np.random.default_rng(4)
    A32 = g.standard_normal((3000, 40)).astype(np.float32)
    spec = P.SketchSpec(256, kind="srht", seed=2)
    out = P.sketch_apply(P.Matrix(dense=torch.from_numpy(A32).cuda()), spec, out_dtype=dt)
    ref = DS.sketch_apply_srht(A32.astype(np.float64), 2, 0, 256, out_dtype=dt)
    assert np.array_equal(host(out), np.asarray(ref, dtype=np.float64))


def test_srht_csr_equals_dense(gpu_lib):
    """CSR data: the sketch of the expanded rows, bitwise."""
    P = gpu_lib
    wl = W.table1_like("w8a", rows=6000)
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d)
    spec = P.SketchSpec(600, kind="srht", seed=8, iter=1)
    out = host(P.sketch_apply(M, spec))
    dense = W.csr_to_dense(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    assert np.array_equal(out, DS.sketch_apply_srht(dense, 8, 1, 600))


@pytest.mark.parametrize("n,d,m", [(1000, 33, 100), (4096, 64, 512), (3, 5, 7), (1, 70, 130),
                                   (20000, 130, 67)])
def test_gaussian_within_bound(gpu_lib, n, d, m):
    P = gpu_lib
    g = np.random.default_rng(n * 3 + d)
    A = g.standard_normal((n, d))
    spec = P.SketchSpec(m, kind="gaussian", seed=12, iter=5)
    out = host(P.sketch_apply(P.Matrix(dense=dev(A)), spec))
    ref = DS.sketch_apply_gaussian(A, 12, 5, m)
    assert np.all(np.abs(out - ref) <= gauss_bound(A, 12, 5, m))


def test_gaussian_float32_and_csr(gpu_lib):
    import torch
    P = gpu_lib
    g = np.random.default_rng(9)
    A32 = g.standard_normal((2500, 48)).astype(np.float32)
    A64 = A32.astype(np.float64)
    spec = P.SketchSpec(96, kind="gaussian", seed=3)
    out = host(P.sketch_apply(P.Matrix(dense=torch.from_numpy(A32).cuda()), spec))
    assert np.all(np.abs(out - DS.sketch_apply_gaussian(A64, 3, 0, 96)) <=
                  gauss_bound(A64, 3, 0, 96))
    wl = W.table1_like("w8a", rows=3000)
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d)
    dense = W.csr_to_dense(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    out = host(P.sketch_apply(M, spec))
    assert np.all(np.abs(out - DS.sketch_apply_gaussian(dense, 3, 0, 96)) <=
                  gauss_bound(dense, 3, 0, 96))


def test_dense_kinds_refuse_hash_adjoint_and_batches(gpu_lib):
    P = gpu_lib
    A = dev(np.ones((10, 3)))
    for kind in ("srht", "gaussian"):
        spec = P.SketchSpec(4, kind=kind)
        with pytest.raises(P.IHSError) as e:
            P.sketch_hash(10, spec)
        assert e.value.code == P.ERR_UNSUPPORTED
        with pytest.raises(P.IHSError) as e:
            P.sketch_apply(P.Matrix(dense=A, row_offsets=[0, 4, 10]), spec)
        assert e.value.code == P.ERR_UNSUPPORTED


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
def test_ihs_with_dense_sketches_matches_oracle(gpu_lib, kind):
    """IHS (Eq.(2)) with the comparison sketches: the iterates against the
    oracle's within the rounding budget (for the Gaussian sketch the budget
    also carries the bound on |dSA| above), and geometric decay."""
    P = gpu_lib
    wl = W.ols_dense(rows=6000, d=40, m=400, iters=8)
    opts = P.options(wl.m, kind=kind, seed=wl.sketch_seed, max_iter=wl.iters)
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0
    xs, Hs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=wl.iters,
                   return_hessians=True, kind=kind)
    apply = DS.sketch_apply_srht if kind == "srht" else DS.sketch_apply_gaussian
    sas = [apply(wl.A, wl.sketch_seed, t, wl.m) for t in range(wl.iters)]
    errs = None if kind == "srht" else [gauss_bound(wl.A, wl.sketch_seed, t, wl.m) / 2
                                        for t in range(wl.iters)]
    bud = RB.ihs_budget(wl.A, wl.b, sas, Hs, xs, sketch_errs=errs)
    hist = host(res.history)[:, 0, :]
    for t in range(wl.iters):
        da = np.linalg.norm(wl.A @ (hist[t] - xs[t + 1]))
        assert da <= bud[t][0], (t, da, bud[t][0])
    xo = O.x_opt(wl.A, wl.b)
    assert O.error_A(wl.A, hist[-1], xo) < 0.5 ** 7 * O.error_A(wl.A, hist[0], xo)
