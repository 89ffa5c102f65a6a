"""GPU parity at the conditioning and widths the measured workloads run at.

The iterates of the library and of the oracle are compared against the
rounding budget of tests/rounding_budget.py: both run the same sketches, so
they differ only by the rounding of their own summation orders and solves,
followed through the IHS error recurrence (Eq.(2), Thm 2.2). At
kappa(A) = 1e5 (kappa(H) about 1e10) that budget is about 1e-5 of
||A x_OPT|| after the first step and falls with the error to about 5e-12;
a step that lost the backward stability of a Cholesky solve (an explicit
inverse applied carelessly, say) leaves it.
"""
import numpy as np
import pytest

import rounding_budget as RB
import workloads as W
from oracle import ihs as O
from oracle import sketch as OS

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.double().cpu().numpy()


def spd(d, g, cond):
    Q, _ = np.linalg.qr(g.standard_normal((d, d)))
    return Q @ np.diag(np.geomspace(1.0, cond, d)) @ Q.T


# ------------------------------------- the step at kappa(H) up to 1e10 ----
@pytest.mark.parametrize("d", [128, 512])
@pytest.mark.parametrize("cond", [1e8, 1e10])
def test_qp_unconstrained_ill_conditioned(gpu_lib, d, cond):
    """From d = 89 on the step applies an explicit inverse of H. Against the
    oracle's Cholesky solve it must stay within the H-norm budget of two
    backward-stable solves: sqrt(dx^T H dx) of the difference."""
    P = gpu_lib
    g = np.random.default_rng(int(d + np.log10(cond)))
    H = spd(d, g, cond)
    gv = g.standard_normal(d)
    x = g.standard_normal(d)
    out = host(P.qp_step(dev(H[None]), dev(gv[None]), dev(x[None])))[0]
    ref = O.qp_step(H, gv, x)
    diff = (out - x) - (ref - x)
    hn = float(np.sqrt(max(diff @ H @ diff, 0.0)))
    bound = RB.h_norm_budget(H, gv)
    step = float(np.sqrt((ref - x) @ H @ (ref - x)))
    assert hn <= bound, (hn, bound, step)
    print("share of the budget used: %.3g (difference %.3g of the step)" % (hn / bound, hn / step))
    assert bound < 1e-3 * step   # the budget itself is far below the step


# ------------------------- the headline conditioning: kappa(A) = 1e5 ----
@pytest.fixture(scope="module")
def headline():
    """The precision workload's recipe on 2^16 rows (A = G diag(sigma) V,
    sigma log-spaced 1 .. 1e-5, d = 512, CountSketch m = 4096): the oracle's
    30 iterates, their budgets and x_OPT."""
    wl = W.precision(rows=1 << 16, d=512, m=4096, iters=30)
    xs, Hs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=30, return_hessians=True)
    sas = [OS.sketch_apply_dense(wl.A, wl.sketch_seed, t, wl.m) for t in range(30)]
    bud = RB.ihs_budget(wl.A, wl.b, sas, Hs, xs)
    del sas, Hs
    return wl, xs, bud, O.x_opt(wl.A, wl.b)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("schedule", ["overlap", "sequential"])
def test_headline_conditioning_iterates_match_oracle(gpu_lib, headline, schedule):
    P = gpu_lib
    wl, xs, bud, xo = headline
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=30, schedule=schedule)
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0 and res.report.iters == 30
    hist = host(res.history)[:, 0, :]
    worst = 0.0
    for t in range(30):
        da = float(np.linalg.norm(wl.A @ (hist[t] - xs[t + 1])))
        assert da <= bud[t][0], (t, da, bud[t][0])
        worst = max(worst, da / bud[t][0])
    print("largest share of the budget used: %.3g" % worst)
    # Thm 2.2's geometric decay takes the prediction-norm error to 1e-10
    assert O.error_A(wl.A, hist[-1], xo) <= 1e-10
    assert O.error_A(wl.A, xs[-1], xo) <= 1e-10


# --------------- the CSR ridge workload at its own width (d = 1024) ----
@pytest.fixture(scope="module", params=[0.5, 3.0], ids=["active", "inactive"])
def ridge_wide(request):
    """The CSR ridge recipe (density 1e-3, Zipf(1.1) columns) at d = 1024,
    m = 8192 on 2^18 rows; radius 0.5 ||x*|| (active ball) and 3 ||x*||
    (inactive: the unconstrained minimiser is inside)."""
    wl = W.ridge_csr(rows=1 << 18, d=1024, m=8192, iters=12, radius_factor=request.param)
    csr = (wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    A = O.csr_matrix(*csr)
    xs, Hs = O.ihs(None, wl.b, wl.m, seed=wl.sketch_seed, iters=wl.iters, constraint="l2",
                   radius=wl.radius, csr=csr, return_hessians=True)
    sas = [OS.sketch_apply_csr(*csr, wl.sketch_seed, t, wl.m) for t in range(wl.iters)]
    bud = RB.ihs_budget(A, wl.b, sas, Hs, xs, "l2", wl.radius)
    del sas, Hs
    return wl, A, xs, bud, O.x_opt(A, wl.b, "l2", wl.radius)


@pytest.mark.timeout(900)
def test_l2_csr_full_width_iterates_match_oracle(gpu_lib, ridge_wide):
    P = gpu_lib
    wl, A, xs, bud, xo = ridge_wide
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l2",
                     radius=wl.radius)
    res = P.solve(M, dev(wl.b), opts, history=True)
    assert res.report.status == 0
    hist = host(res.history)[:, 0, :]
    active = np.linalg.norm(xo) > wl.radius * (1 - 1e-9)
    assert active == (wl.radius < np.linalg.norm(wl.x_star))
    worst = 0.0
    for t in range(wl.iters):
        assert np.linalg.norm(hist[t]) <= wl.radius * (1 + 1e-12)
        da = float(np.linalg.norm(A @ (hist[t] - xs[t + 1])))
        de = float(np.linalg.norm(hist[t] - xs[t + 1]))
        assert da <= bud[t][0], (t, da, bud[t][0])
        assert de <= bud[t][1], (t, de, bud[t][1])
        worst = max(worst, da / bud[t][0], de / bud[t][1])
    print("largest share of the budget used: %.3g" % worst)
    assert O.error_A(A, hist[-1], xo) < 1e-3 * O.error_A(A, hist[0], xo)
