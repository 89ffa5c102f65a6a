"""The outer loop's tolerance stop: after step t the solve ends when every
problem's step length in the prediction norm, sqrt(dx^T H_t dx), is at most
tol (Thm 2.2: Theta(log 1/eps) steps reach an eps-solution). The decision is
taken on the device, so a stopped solve must equal, bit for bit, a solve of
exactly the reported number of steps."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.double().cpu().numpy()


def _problem(kind):
    if kind == "ridge":
        wl = W.ridge_csr(rows=1 << 15, d=128, density=8e-3, m=1024, radius_factor=0.5)
        return wl, dict(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                        n=wl.n, d=wl.d), "l2", wl.radius
    if kind == "lasso":
        wl = W.lasso_dense(rows=20000, d=64, m=512)
        return wl, dict(dense=dev(wl.A)), "l1", wl.radius
    if kind == "penalty":
        wl = W.lasso_dense(rows=6000, d=24, m=192, penalty=40.0)
        return wl, dict(dense=dev(wl.A)), "l1_penalty", wl.radius
    if kind == "ragged":
        wl = W.batch_ragged(num=5, n_lo=2000, n_hi=9000, d=64)
        return wl, dict(dense=dev(wl.A), row_offsets=wl.row_offsets), "none", 0.0
    wl = W.ols_dense(rows=20000, d=50 if kind == "ols" else 128, m=500 if kind == "ols" else 1280)
    return wl, dict(dense=dev(wl.A)), "none", 0.0


@pytest.mark.parametrize("kind,schedule", [
    ("ols", "overlap"), ("ols", "sequential"), ("ols128", "overlap"), ("ols128", "sequential"),
    ("lasso", "overlap"), ("lasso", "sequential"), ("ridge", "overlap"),
    ("penalty", "sequential"), ("ragged", "overlap")])
def test_tol_stop_equals_fixed_step_count(gpu_lib, kind, schedule):
    P = gpu_lib
    wl, mat, cons, radius = _problem(kind)
    M = P.Matrix(**mat)
    b = dev(wl.b)
    N = 40
    # a tolerance the solve meets part-way: 1e-6 of the first step's length
    # (a one-step solve with a tolerance it cannot meet records that length)
    first = P.solve(M, b, P.options(wl.m, seed=wl.sketch_seed, max_iter=1, constraint=cons,
                                    radius=radius, schedule="sequential", tol=1e-300),
                    raise_on_error=False)
    assert first.report.status == P.ERR_NOT_CONVERGED and first.report.last_step > 0
    tol = 1e-6 * first.report.last_step
    o = P.options(wl.m, seed=wl.sketch_seed, max_iter=N, constraint=cons, radius=radius,
                  schedule=schedule, tol=tol)
    stopped = P.solve(M, b, o, history=True)
    k = stopped.report.iters
    assert stopped.report.status == 0 and 1 < k < N, k
    assert stopped.report.failed_iter == -1
    assert stopped.report.last_step <= tol or M.batch > 1
    fixed = P.solve(M, b, P.options(wl.m, seed=wl.sketch_seed, max_iter=k, constraint=cons,
                                    radius=radius, schedule=schedule), history=True)
    assert np.array_equal(host(stopped.x), host(fixed.x))
    h = host(stopped.history)
    assert np.array_equal(h[:k], host(fixed.history))
    for t in range(k, N):   # later rows repeat the final iterate
        assert np.array_equal(h[t], h[k - 1])
    assert stopped.report.objective == fixed.report.objective


def test_tol_not_met_returns_not_converged(gpu_lib):
    """A tolerance below what max_iter steps reach: IHS_ERR_NOT_CONVERGED,
    every step taken, x equal to the fixed-count solve."""
    P = gpu_lib
    wl, mat, _, _ = _problem("ols")
    M = P.Matrix(**mat)
    b = dev(wl.b)
    o = P.options(wl.m, seed=wl.sketch_seed, max_iter=5, tol=1e-300)
    res = P.solve(M, b, o, raise_on_error=False)
    assert res.report.status == P.ERR_NOT_CONVERGED
    assert res.report.iters == 5 and res.report.failed_iter == -1
    fixed = P.solve(M, b, P.options(wl.m, seed=wl.sketch_seed, max_iter=5))
    assert np.array_equal(host(res.x), host(fixed.x))
    with pytest.raises(P.IHSError) as e:
        P.solve(M, b, o)
    assert e.value.code == P.ERR_NOT_CONVERGED
