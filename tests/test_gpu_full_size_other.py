"""Sampled parity at the full sizes of the lasso and CSR-ridge workloads, in
the launch configurations the benchmark times (its per-row timings): the
lasso matrix 2^20 x 256 (rows ~ N(0, Sigma), generated on the device as the
benchmark generates it) with CountSketch and with the SJLT (s = 4), both at
m = 4096, and the Zipf CSR matrix 2^22 x 1024 at density 1e-3 with m = 8192.

  * the hash (Sec. 2) of every (row, block) pair, bit-exact;
  * S A on sampled sketch rows, bit-exact: the rows of each sampled bucket
    are fetched and summed on the host in ascending row order with their
    signs, and an SJLT block's sum is scaled by 1/sqrt(s) afterwards (the
    sequential definition the kernels follow)."""
import numpy as np
import pytest

import workloads as W
from oracle import sketch as OS

pytestmark = pytest.mark.gpu


def picks_for(m, seed):
    g = np.random.default_rng(seed)
    return np.concatenate([[0, m - 1], g.choice(np.arange(1, m - 1), 6, replace=False)])


@pytest.fixture(scope="module")
def lasso(gpu_lib):
    import torch
    wl = W.lasso_dense(backend="torch", device="cuda")
    torch.cuda.synchronize()
    yield wl
    del wl
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,s", [("countsketch", 1), ("sjlt", 4)])
def test_lasso_full_size_hash_and_sampled_rows(gpu_lib, lasso, kind, s):
    import torch
    P, wl = gpu_lib, lasso
    n, d, m, it = wl.n, wl.d, 4096, 2
    spec = P.SketchSpec(m, s, kind, seed=wl.sketch_seed, iter=it)
    b, sg = P.sketch_hash(n, spec)
    rb, rs = OS.sketch_hash(wl.sketch_seed, it, n, m, s)
    assert np.array_equal(b.cpu().numpy(), rb)
    assert np.array_equal(sg.cpu().numpy(), rs)
    SA = P.sketch_apply(P.Matrix(dense=wl.A), spec)
    picks = picks_for(m, 20 + s)
    got = SA[torch.as_tensor(picks, device="cuda")].cpu().numpy()
    m_blk = m // s
    for q, r in enumerate(picks):
        k = r // m_blk                                   # the block of sketch row r
        rows = np.nonzero(rb[:, k] == r)[0]              # ascending row order
        assert len(rows) > 0, r
        Ar = wl.A[torch.as_tensor(rows, device="cuda")].cpu().numpy()
        acc = np.zeros(d)
        for i, row in enumerate(rows):
            acc = acc + float(rs[row, k]) * Ar[i]
        if s > 1:
            acc = acc * (1.0 / np.sqrt(s))
        assert np.array_equal(got[q], acc), (kind, r)


def test_csr_full_size_hash_and_sampled_rows(gpu_lib):
    import torch
    P = gpu_lib
    wl = W.ridge_csr()
    n, d, m, it = wl.n, wl.d, 8192, 4
    M = P.Matrix(row_ptr=torch.from_numpy(wl.indptr).cuda(),
                 col_idx=torch.from_numpy(wl.indices).cuda(),
                 values=torch.from_numpy(wl.data).cuda(), n=n, d=d)
    spec = P.SketchSpec(m, 1, seed=wl.sketch_seed, iter=it)
    b, sg = P.sketch_hash(n, spec)
    rb, rs = OS.sketch_hash(wl.sketch_seed, it, n, m, 1)
    assert np.array_equal(b.cpu().numpy(), rb)
    assert np.array_equal(sg.cpu().numpy(), rs)
    SA = P.sketch_apply(M, spec)
    picks = picks_for(m, 30)
    got = SA[torch.as_tensor(picks, device="cuda")].cpu().numpy()
    for q, r in enumerate(picks):
        rows = np.nonzero(rb[:, 0] == r)[0]
        assert len(rows) > 0, r
        acc = np.zeros(d)
        for row in rows:                                  # ascending; columns distinct
            lo, hi = wl.indptr[row], wl.indptr[row + 1]
            cols = wl.indices[lo:hi]
            acc[cols] = acc[cols] + float(rs[row, 0]) * wl.data[lo:hi]
        assert np.array_equal(got[q], acc), r
    del M, SA
    torch.cuda.empty_cache()
