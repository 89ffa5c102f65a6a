"""Parity at the full size of the precision workload: A = G diag(sigma) V,
2^22 x 512 float64, condition number 1e5, CountSketch with m = 4096 (the
configuration the benchmark times), generated on the device as the benchmark
generates it, and run in the launch configuration the benchmark uses.

The oracle cannot take a 16 GiB matrix in seconds, so outputs are checked
where it can compute them one by one:
  * the hash (Sec. 2) for every one of the 2^22 rows, bit-exact;
  * S A (Sec. 2) on sampled sketch rows: the rows of each sampled bucket are
    fetched from the device and summed in ascending row order on the host, which
    must reproduce the kernel's row bit for bit;
  * the gradient side of Eq.(2) at a sparse x on sampled columns, against the
    exactly rounded sum (math.fsum) within the forward-error bound of a length-n
    float64 sum, and the residual r = b - A x on every row;
  * the overlapped solver schedules against the sequential one over three steps
    (a property: the same sketches give the same factors bit for bit; the
    gradient is summed in another row order, so iterates agree to rounding,
    amplified by at most the condition number of H)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sketch as OS

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def full(gpu_lib):
    import torch
    wl = W.precision(backend="torch", device="cuda")
    torch.cuda.synchronize()
    yield wl
    del wl
    torch.cuda.empty_cache()


def test_full_size_hash_bit_exact(gpu_lib, full):
    P, wl = gpu_lib, full
    spec = P.SketchSpec(wl.m, 1, seed=wl.sketch_seed, iter=3)
    b, sg = P.sketch_hash(wl.n, spec)
    rb, rs = OS.sketch_hash(wl.sketch_seed, 3, wl.n, wl.m, 1)
    assert np.array_equal(b.cpu().numpy(), rb)
    assert np.array_equal(sg.cpu().numpy(), rs)


def test_full_size_sketch_sampled_rows_bit_exact(gpu_lib, full):
    import torch
    P, wl = gpu_lib, full
    n, d, m, it = wl.n, wl.d, wl.m, 5
    SA = P.sketch_apply(P.Matrix(dense=wl.A), P.SketchSpec(m, 1, seed=wl.sketch_seed, iter=it))
    bucket, sign = OS.sketch_hash(wl.sketch_seed, it, n, m, 1)
    g = np.random.default_rng(10)
    picks = np.concatenate([[0, m - 1], g.choice(np.arange(1, m - 1), 6, replace=False)])
    got = SA[torch.as_tensor(picks, device="cuda")].cpu().numpy()
    for k, r in enumerate(picks):
        rows = np.nonzero(bucket[:, 0] == r)[0]          # ascending row order
        Ar = wl.A[torch.as_tensor(rows, device="cuda")].cpu().numpy()
        acc = np.zeros(d)
        for i, row in enumerate(rows):
            acc = acc + float(sign[row, 0]) * Ar[i]
        assert len(rows) > 0, r
        assert np.array_equal(got[k], acc), r


def test_full_size_gradient_sampled_columns(gpu_lib, full):
    import torch
    P, wl = gpu_lib, full
    n, d = wl.n, wl.d
    k1, k2, c1, c2 = 3, 400, 0.75, -1.25
    x = torch.zeros(1, d, dtype=torch.float64, device="cuda")
    x[0, k1], x[0, k2] = c1, c2
    g, r, f = P.gradient(P.Matrix(dense=wl.A), wl.b, x, want_r=True)
    torch.cuda.synchronize()
    bh = wl.b.cpu().numpy()
    a1 = wl.A[:, k1].cpu().numpy()
    a2 = wl.A[:, k2].cpu().numpy()
    mag = np.abs(bh) + np.abs(a1 * c1) + np.abs(a2 * c2)   # bounds |r_i| and its terms
    # residual: three terms per row (the zero coordinates add exact zeros)
    rh = r.cpu().numpy()
    r_ref = bh - (a1 * c1 + a2 * c2)
    assert np.all(np.abs(rh - r_ref) <= 6 * U * mag)
    gh = g.cpu().numpy()[0]
    for j in (0, k1, 255, k2, d - 1):
        aj = a1 if j == k1 else a2 if j == k2 else wl.A[:, j].cpu().numpy()
        terms = np.concatenate([aj * bh, -(aj * a1) * c1, -(aj * a2) * c2])
        exact = math.fsum(terms)
        bound = (n + 8) * U * float(np.sum(np.abs(aj) * mag)) * 1.01
        assert abs(gh[j] - exact) <= bound, (j, gh[j], exact, bound)
    f_exact = 0.5 * math.fsum(r_ref * r_ref)
    assert abs(float(f[0]) - f_exact) <= (n + 8) * U * 0.5 * float(np.sum(mag * mag)) * 1.01


def test_full_size_overlapped_schedules_match_sequential(gpu_lib, full):
    import torch
    P, wl = gpu_lib, full
    M = P.Matrix(dense=wl.A)
    runs = {}
    for sched in ("sequential", "overlap", "overlap2"):
        o = P.options(wl.m, seed=wl.sketch_seed, max_iter=3, schedule=sched)
        res = P.solve(M, wl.b, o, history=True, factors=True)
        runs[sched] = (res.history.cpu().numpy(), res.factors.cpu().numpy())
    torch.cuda.synchronize()
    hs, fs = runs["sequential"]
    for sched in ("overlap", "overlap2"):
        h, f = runs[sched]
        assert np.array_equal(f, fs), sched
        for t in range(3):
            assert np.linalg.norm(h[t] - hs[t]) <= 1e-6 * np.linalg.norm(hs[t]), (sched, t)
