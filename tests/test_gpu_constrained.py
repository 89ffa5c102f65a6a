"""GPU parity of the constrained steps of Eq.(2) (l1 and l2 balls of Eq.(1))
and of IHS on the constrained problems, against the oracle.

The QP solution is unique for a positive definite H, so the GPU's inner
iterates (a different step size, restart rule and projection order than the
oracle's) are not compared; only the solution is. Both sides end on the
exact solution of the identified face (l1: the KKT system of the support and
signs; l2: the root of the secular equation), so they may differ only by
the rounding of forming c = H x^t + g and of that final solve. The
tolerances are the rounding budgets of tests/rounding_budget.py (for the
library's conjugate-gradient polish of large supports, its residual test is
added); the IHS iterates are compared against the same budget carried
through the steps. Every l1 QP must end on a KKT-certified polish
(report.qp_unpolished == 0): a converged first-order iterate the polish did
not certify would be accurate only to the inner stopping test."""
import numpy as np
import pytest

import rounding_budget as RB
import workloads as W
from conftest import INVERSE_MIN_D
from oracle import ihs as O
from oracle import sketch as OS

# the library's conjugate-gradient polish stops at this relative residual
CG_TOL = 1e-15
U = 2.0 ** -53


def kkt_tol(H, c, x):
    """Bound on the scaled KKT residual of an exact face solution: the
    residual c - H x is formed with length-d dot products (error at most
    gamma_d (|H||x| + |c|), with gamma_d <= 1.01 d u), and the polish solves
    the face to rounding or to the conjugate-gradient residual CG_TOL."""
    d = len(c)
    scale = max(1.0, np.abs(c).max())
    return (2.02 * d * U + 2 * CG_TOL) * (np.abs(H) @ np.abs(x) + np.abs(c)).max() / scale

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.double().cpu().numpy()


def spd(d, g, cond):
    Q, _ = np.linalg.qr(g.standard_normal((d, d)))
    return Q @ np.diag(np.geomspace(1.0, cond, d)) @ Q.T


def unconstrained_min(H, g, x):
    return x + np.linalg.solve(H, g)


def kkt_l1_residual(H, c, x, tau):
    """Max violation of the l1-ball KKT conditions at x (scaled)."""
    grad = c - H @ x
    S = x != 0
    if not S.any():
        return np.inf
    mu = float(np.mean(grad[S] * np.sign(x[S])))
    scale = max(1.0, np.abs(c).max())
    on = np.abs(grad[S] - mu * np.sign(x[S])).max() / scale
    off = max(0.0, (np.abs(grad[~S]).max() - mu) / scale) if (~S).any() else 0.0
    feas = max(0.0, np.abs(x).sum() - tau) / tau
    return max(on, off, feas, max(0.0, -mu / scale))


# ------------------------------------------------------------ l1 ball ----
@pytest.mark.parametrize("d,batch,frac,cond", [
    (8, 1, 0.5, 10.0), (50, 2, 0.3, 1e2), (64, 3, 0.6, 1e2), (130, 1, 0.5, 1e2),
    (256, 1, 0.5, 1e2), (256, 1, 0.97, 10.0), (1000, 1, 0.5, 10.0), (1, 1, 0.5, 1.0),
    (97, 2, 0.05, 1e3)])
def test_qp_l1_matches_oracle(gpu_lib, d, batch, frac, cond):
    P = gpu_lib
    g = np.random.default_rng(1000 + d)
    Hs = np.stack([spd(d, g, cond) for _ in range(batch)])
    gs = g.standard_normal((batch, d))
    xs = 0.1 * g.standard_normal((batch, d))
    # one radius for the batch, active for every problem
    tau = frac * min(np.abs(unconstrained_min(Hs[p], gs[p], xs[p])).sum() for p in range(batch))
    out, rep = P.qp_step(dev(Hs), dev(gs), dev(xs), constraint="l1", radius=tau,
                         want_report=True)
    out = host(out)
    assert rep.status == 0 and rep.qp_unpolished == 0
    for p in range(batch):
        ref = O.qp_step(Hs[p], gs[p], xs[p], "l1", tau)
        assert np.abs(out[p]).sum() <= tau * (1 + 1e-12)
        assert np.array_equal(np.sign(out[p]), np.sign(ref)), p   # the same face
        bound = RB.qp_budget(Hs[p], gs[p], xs[p], ref, "l1", tau, cg_tol=CG_TOL)
        assert np.linalg.norm(out[p] - ref) <= bound, (p, np.linalg.norm(out[p] - ref), bound)
        print("share of the budget used: %.3g" % (np.linalg.norm(out[p] - ref) / bound))
        c = Hs[p] @ xs[p] + gs[p]
        assert kkt_l1_residual(Hs[p], c, out[p], tau) <= kkt_tol(Hs[p], c, out[p])


@pytest.mark.parametrize("d", [77, 200])
def test_qp_l1_inactive_ball_is_the_unconstrained_step(gpu_lib, d):
    """An inactive ball returns the unconstrained step: bit for bit where the
    ball step forms it the way the unconstrained step does (every width for
    the l2 ball; below d = 89 for the l1 ball, whose minimiser always comes
    from the triangular solves), to rounding otherwise."""
    P = gpu_lib
    g = np.random.default_rng(7)
    H, gv, x = spd(d, g, 1e2)[None], g.standard_normal((1, d)), g.standard_normal((1, d))
    free = host(P.qp_step(dev(H), dev(gv), dev(x)))
    tau = 10 * np.abs(free).sum()
    for cons in ("l1", "l2"):
        out = host(P.qp_step(dev(H), dev(gv), dev(x), constraint=cons, radius=tau))
        if cons == "l2" or d < INVERSE_MIN_D:
            assert np.array_equal(out, free), cons
        else:
            assert np.linalg.norm(out - free) <= 1e-12 * 1e2 * np.linalg.norm(free - x), cons


def test_qp_l1_not_converged_keeps_iterate(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(8)
    d = 300
    H, gv = spd(d, g, 1e3)[None], g.standard_normal((1, d))
    x = 0.01 * g.standard_normal((1, d))
    tau = 0.5 * np.abs(unconstrained_min(H[0], gv[0], x[0])).sum()
    with pytest.raises(P.IHSError) as e:
        P.qp_step(dev(H), dev(gv), dev(x), constraint="l1", radius=tau, qp_max_inner=2)
    assert e.value.code == P.ERR_NOT_CONVERGED


def test_qp_l1_projection_special_case(gpu_lib):
    """H = I: the minimiser of 1/2||x||^2 - c^T x over the ball is the
    Euclidean projection of c, fixed here by a hand-checkable case."""
    P = gpu_lib
    H = np.eye(4)[None]
    c = np.array([[3.0, -1.0, 0.5, 0.0]])
    out = host(P.qp_step(dev(H), dev(c), dev(np.zeros((1, 4))), constraint="l1", radius=2.0))
    # threshold theta = 1: the largest magnitude alone exceeds it, 3 - 1 = 2
    np.testing.assert_allclose(out[0], [2.0, 0.0, 0.0, 0.0], atol=1e-14)


# ------------------------------------------------------------ l2 ball ----
@pytest.mark.parametrize("d,batch,frac,cond", [
    (8, 1, 0.5, 10.0), (50, 3, 0.3, 1e2), (100, 1, 0.9, 1e3), (513, 1, 0.5, 1e2),
    (1024, 1, 0.2, 1e2), (1, 1, 0.5, 1.0), (200, 2, 0.999, 1e2)])
def test_qp_l2_matches_oracle(gpu_lib, d, batch, frac, cond):
    P = gpu_lib
    g = np.random.default_rng(2000 + d)
    Hs = np.stack([spd(d, g, cond) for _ in range(batch)])
    gs = g.standard_normal((batch, d))
    xs = 0.1 * g.standard_normal((batch, d))
    r = frac * min(np.linalg.norm(unconstrained_min(Hs[p], gs[p], xs[p])) for p in range(batch))
    out = host(P.qp_step(dev(Hs), dev(gs), dev(xs), constraint="l2", radius=r))
    for p in range(batch):
        ref = O.qp_step(Hs[p], gs[p], xs[p], "l2", r)
        assert np.linalg.norm(out[p]) <= r * (1 + 1e-12)
        bound = RB.qp_budget(Hs[p], gs[p], xs[p], ref, "l2", r)
        assert np.linalg.norm(out[p] - ref) <= bound, (p, np.linalg.norm(out[p] - ref), bound)
        print("share of the budget used: %.3g" % (np.linalg.norm(out[p] - ref) / bound))


@pytest.mark.parametrize("d", [40, 100])
def test_qp_l2_mixed_batch_and_identity(gpu_lib, d):
    """H = I gives x = c min(1, r/||c||) (closed form); a batch where one
    problem's ball is inactive and the other's active. d = 100 takes the cold
    start through the explicit inverse, d = 40 through the triangular solves."""
    P = gpu_lib
    g = np.random.default_rng(11)
    c = np.stack([0.1 * g.standard_normal(d), 10.0 * g.standard_normal(d)])
    H = np.stack([np.eye(d), np.eye(d)])
    out = host(P.qp_step(dev(H), dev(c), dev(np.zeros((2, d))), constraint="l2", radius=1.0))
    for p in range(2):
        want = c[p] * min(1.0, 1.0 / np.linalg.norm(c[p]))
        np.testing.assert_allclose(out[p], want, rtol=1e-12, atol=1e-15)


# --------------------------------------------------- constrained IHS ----
def oracle_run(A, b, m, s, seed, iters, constraint, radius, csr=None):
    """The oracle's iterates, their rounding budgets and A as an operator."""
    xs, Hs = O.ihs(None if csr else A, b, m, s=s, seed=seed, iters=iters,
                   constraint=constraint, radius=radius, csr=csr, return_hessians=True)
    if csr is not None:
        sas = [OS.sketch_apply_csr(*csr, seed, t, m, s) for t in range(iters)]
        A = O.csr_matrix(*csr)
    else:
        sas = [OS.sketch_apply_dense(A, seed, t, m, s) for t in range(iters)]
    return xs, RB.ihs_budget(A, b, sas, Hs, xs, constraint, radius), A


def assert_within_budget(A, hist, xs, bud, what=""):
    worst = 0.0
    for t in range(len(bud)):
        de = float(np.linalg.norm(hist[t] - xs[t + 1]))
        da = float(np.linalg.norm(A @ (hist[t] - xs[t + 1])))
        assert de <= bud[t][1] and da <= bud[t][0], (what, t, de, bud[t][1], da, bud[t][0])
        worst = max(worst, de / bud[t][1], da / bud[t][0])
    print("largest share of the budget used: %.3g" % worst)


@pytest.mark.parametrize("kind,s", [("countsketch", 1), ("sjlt", 4)])
def test_ihs_l1_lasso_iterates_match_oracle(gpu_lib, kind, s):
    P = gpu_lib
    wl = W.lasso_dense(rows=40000, d=64, m=1024, sketch=kind, iters=6)
    opts = P.options(wl.m, s=s, kind=kind, seed=wl.sketch_seed, max_iter=wl.iters,
                     constraint="l1", radius=wl.radius)
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0 and res.report.qp_unpolished == 0
    xs, bud, _ = oracle_run(wl.A, wl.b, wl.m, s, wl.sketch_seed, wl.iters, "l1", wl.radius)
    hist = host(res.history)[:, 0, :]
    for t in range(wl.iters):
        assert np.abs(hist[t]).sum() <= wl.radius * (1 + 1e-12)
    assert_within_budget(wl.A, hist, xs, bud, kind)
    xo = O.x_opt(wl.A, wl.b, "l1", wl.radius)
    assert O.error_A(wl.A, hist[-1], xo) < 0.05 * O.error_A(wl.A, hist[0], xo)


def test_ihs_l1_lasso_full_width(gpu_lib):
    """The lasso shape at d = 256, m = 4096 on a row-scaled sample: the
    iterates match the oracle and the error in the prediction norm falls."""
    P = gpu_lib
    wl = W.lasso_dense(rows=1 << 16, d=256, m=4096, iters=4)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l1",
                     radius=wl.radius)
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0 and res.report.qp_unpolished == 0
    xs, bud, _ = oracle_run(wl.A, wl.b, wl.m, 1, wl.sketch_seed, wl.iters, "l1", wl.radius)
    hist = host(res.history)[:, 0, :]
    assert_within_budget(wl.A, hist, xs, bud)


def test_ihs_l2_csr_iterates_match_oracle(gpu_lib):
    P = gpu_lib
    wl = W.ridge_csr(rows=1 << 15, d=128, density=8e-3, m=1024, iters=6, radius_factor=0.5)
    A = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l2",
                     radius=wl.radius)
    res = P.solve(A, dev(wl.b), opts, history=True)
    assert res.report.status == 0
    csr = (wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    xs, bud, Asp = oracle_run(None, wl.b, wl.m, 1, wl.sketch_seed, wl.iters, "l2", wl.radius,
                              csr=csr)
    hist = host(res.history)[:, 0, :]
    for t in range(wl.iters):
        assert np.linalg.norm(hist[t]) <= wl.radius * (1 + 1e-12)
    assert_within_budget(Asp, hist, xs, bud)
    xo = O.x_opt(Asp, wl.b, "l2", wl.radius)
    assert O.error_A(Asp, hist[-1], xo) < 0.1 * O.error_A(Asp, hist[0], xo)


def test_ihs_l2_csr_bf16_gram_converges(gpu_lib):
    """CSR with the BF16 Gram (FP32 accumulation): the outer loop still
    drives the error down on a well-conditioned Zipf problem."""
    P = gpu_lib
    wl = W.ridge_csr(rows=1 << 15, d=128, density=8e-3, m=1024, iters=10, radius_factor=0.5)
    A = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d)
    csr = (wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    Asp = O.csr_matrix(*csr)
    xo = O.x_opt(Asp, wl.b, "l2", wl.radius)
    errs = {}
    for gin, gacc in (("float64", "float64"), ("bfloat16", "float32")):
        opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l2",
                         radius=wl.radius, gram_in=gin, gram_acc=gacc)
        res = P.solve(A, dev(wl.b), opts)
        assert res.report.status == 0
        errs[gin] = O.error_A(Asp, host(res.x)[0], xo)
    assert errs["float64"] < 1e-2
    assert errs["bfloat16"] < 3 * errs["float64"] + 1e-6


# -------------------------------------------- l1 penalty (Sec. 3 LASSO) ----
def kkt_l1_penalty_residual(H, c, x, lam):
    """Max violation (scaled) of the optimality conditions of
    1/2 x^T H x - c^T x + lam ||x||_1 at x."""
    grad = c - H @ x
    S = x != 0
    scale = max(1.0, np.abs(c).max())
    on = np.abs(grad[S] - lam * np.sign(x[S])).max() / scale if S.any() else 0.0
    off = max(0.0, (np.abs(grad[~S]).max() - lam) / scale) if (~S).any() else 0.0
    return max(on, off)


@pytest.mark.parametrize("d,batch,frac,cond", [
    (8, 1, 0.3, 10.0), (50, 2, 0.2, 1e2), (64, 3, 0.5, 1e2), (256, 1, 0.1, 1e2),
    (600, 1, 0.3, 10.0), (1, 1, 0.5, 1.0), (97, 2, 0.01, 1e3)])
def test_qp_l1_penalty_matches_oracle(gpu_lib, d, batch, frac, cond):
    P = gpu_lib
    g = np.random.default_rng(3000 + d)
    Hs = np.stack([spd(d, g, cond) for _ in range(batch)])
    gs = g.standard_normal((batch, d))
    xs = 0.1 * g.standard_normal((batch, d))
    # one weight for the batch: a fraction of the smallest max |c|
    lam = frac * min(np.abs(Hs[p] @ xs[p] + gs[p]).max() for p in range(batch))
    out, rep = P.qp_step(dev(Hs), dev(gs), dev(xs), constraint="l1_penalty", radius=lam,
                         want_report=True)
    out = host(out)
    assert rep.status == 0 and rep.qp_unpolished == 0
    for p in range(batch):
        ref = O.qp_step(Hs[p], gs[p], xs[p], "l1_penalty", lam)
        assert np.array_equal(np.sign(out[p]), np.sign(ref)), p   # the same face
        bound = RB.qp_budget(Hs[p], gs[p], xs[p], ref, "l1_penalty", lam, cg_tol=CG_TOL)
        assert np.linalg.norm(out[p] - ref) <= bound, (p, np.linalg.norm(out[p] - ref), bound)
        print("share of the budget used: %.3g" % (np.linalg.norm(out[p] - ref) / bound))
        c = Hs[p] @ xs[p] + gs[p]
        assert kkt_l1_penalty_residual(Hs[p], c, out[p], lam) <= kkt_tol(Hs[p], c, out[p])


def test_qp_l1_penalty_special_cases(gpu_lib):
    """H = I gives the soft threshold of c (hand-checkable values); a weight at
    or above max |c| gives exactly 0; a zero weight gives the unconstrained step."""
    P = gpu_lib
    H = np.eye(5)[None]
    c = np.array([[3.0, -2.5, 0.4, -0.1, 1.0]])
    out = host(P.qp_step(dev(H), dev(c), dev(np.zeros((1, 5))), constraint="l1_penalty",
                         radius=1.0))
    np.testing.assert_allclose(out[0], [2.0, -1.5, 0.0, 0.0, 0.0], atol=1e-14)
    g = np.random.default_rng(31)
    d = 40
    Hr, gv, x = spd(d, g, 1e2)[None], g.standard_normal((1, d)), 0.1 * g.standard_normal((1, d))
    lam = np.abs(Hr[0] @ x[0] + gv[0]).max()
    out = host(P.qp_step(dev(Hr), dev(gv), dev(x), constraint="l1_penalty", radius=lam))
    assert np.array_equal(out, np.zeros((1, d)))
    free = host(P.qp_step(dev(Hr), dev(gv), dev(x)))
    out = host(P.qp_step(dev(Hr), dev(gv), dev(x), constraint="l1_penalty", radius=0.0))
    assert np.linalg.norm(out - free) <= 1e-10 * np.linalg.norm(free)


def test_ihs_l1_penalty_iterates_match_oracle(gpu_lib):
    P = gpu_lib
    wl = W.lasso_dense(rows=6000, d=24, m=192, penalty=40.0)
    for kind, s in (("countsketch", 1), ("sjlt", 4)):
        opts = P.options(wl.m, s=s, kind=kind, seed=wl.sketch_seed, max_iter=10,
                         constraint="l1_penalty", radius=wl.radius)
        res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
        assert res.report.status == 0 and res.report.qp_unpolished == 0
        hist = host(res.history)[:, 0]
        xs, bud, _ = oracle_run(wl.A, wl.b, wl.m, s, wl.sketch_seed, 10, "l1_penalty",
                                wl.radius)
        assert_within_budget(wl.A, hist, xs, bud, kind)
        xo = O.x_opt(wl.A, wl.b, "l1_penalty", wl.radius)
        assert O.error_A(wl.A, hist[-1], xo) < 1e-7, kind


@pytest.mark.parametrize("lam", [2.0, 10.0])
def test_ihs_l1_penalty_inverse_polish_matches_oracle(gpu_lib, lam):
    """From the width at which the overlapped schedule forms H_t^{-1} beside
    the pass, the penalised step polishes a face whose complement N is the
    smaller set through that inverse: (H_SS)^{-1} is the Schur complement of
    G_NN in G = H^{-1}. At lambda 2 and 10 the minimiser keeps 113 and 67 of
    128 coordinates. Both schedules' iterates (the sequential one polishes by
    conjugate gradients on H_SS) stay within the oracle's rounding budget."""
    P = gpu_lib
    wl = W.lasso_dense(rows=20000, d=128, m=1024, iters=6, penalty=lam)
    assert wl.d >= INVERSE_MIN_D
    xs, bud, _ = oracle_run(wl.A, wl.b, wl.m, 1, wl.sketch_seed, 6, "l1_penalty", wl.radius)
    M = P.Matrix(dense=dev(wl.A))
    for sched in ("overlap", "sequential"):
        o = P.options(wl.m, seed=wl.sketch_seed, max_iter=6, constraint="l1_penalty",
                      radius=wl.radius, schedule=sched)
        r = P.solve(M, dev(wl.b), o, history=True)
        assert r.report.status == 0 and r.report.qp_unpolished == 0, sched
        assert_within_budget(wl.A, host(r.history)[:, 0], xs, bud, sched)
    assert int((xs[-1] != 0).sum()) > wl.d // 2


@pytest.mark.parametrize("lam", [20.0, 500.0])
def test_ihs_l1_penalty_inverse_polish_ragged_batch(gpu_lib, lam):
    """The same polish through each problem's own H_t^{-1} in a ragged batch
    (three problems of 7471, 6726 and 5733 rows, d = 128). At lambda 20 the
    minimisers keep 128, 128 and 126 coordinates (an empty complement: the
    face solve is two products with H^{-1}); at 500, 119, 117 and 121. Every
    problem's iterates against the oracle's within the rounding budget."""
    P = gpu_lib
    wl = W.batch_ragged(num=3, n_lo=3000, n_hi=8000, d=128, m=1280, iters=6)
    assert wl.d >= INVERSE_MIN_D
    offs = wl.row_offsets
    o = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l1_penalty",
                  radius=lam)
    res = P.solve(P.Matrix(dense=dev(wl.A), row_offsets=offs), dev(wl.b), o, history=True)
    assert res.report.status == 0 and res.report.qp_unpolished == 0
    hist = host(res.history)
    for p in range(wl.batch):
        Ap, bp = wl.A[offs[p]:offs[p + 1]], wl.b[offs[p]:offs[p + 1]]
        x = np.zeros(wl.d)
        xs, sas, Hs = [x.copy()], [], []
        for t in range(wl.iters):
            SA = OS.sketch_apply_dense(Ap, wl.sketch_seed, t, wl.m, 1, problem=p)
            H = SA.T @ SA
            _, gr, _ = O.gradient(Ap, bp, x)
            x = O.qp_step(H, gr, x, "l1_penalty", lam)
            xs.append(x.copy())
            sas.append(SA)
            Hs.append(H)
        assert int((xs[-1] != 0).sum()) > wl.d // 2
        bud = RB.ihs_budget(Ap, bp, sas, Hs, xs, "l1_penalty", lam)
        for t in range(wl.iters):
            dx = hist[t, p] - xs[t + 1]
            assert np.linalg.norm(Ap @ dx) <= bud[t][0], (p, t, np.linalg.norm(Ap @ dx),
                                                         bud[t][0])
            assert np.linalg.norm(dx) <= bud[t][1], (p, t)


def test_ihs_l1_penalty_full_size_kkt(gpu_lib):
    """The penalised LASSO of the experiments (lambda = 5) at the full lasso
    shape (2^20 x 256, CountSketch m = 4096): after 20 steps the iterate meets
    the optimality conditions of the full problem, |A^T (b - A x)|_j <= lambda
    off the support and = lambda sign(x_j) on it, to a relative 1e-6 of
    max |A^T b| (a property that holds at any size; A^T r formed in float64 by
    torch)."""
    import torch
    P = gpu_lib
    wl = W.lasso_dense(backend="torch", device="cuda", penalty=5.0)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l1_penalty",
                     radius=wl.radius)
    x = P.solve(P.Matrix(dense=wl.A), wl.b, opts).x[0]
    grad = (wl.A.T @ (wl.b - wl.A @ x)).cpu().numpy()
    scale = float((wl.A.T @ wl.b).abs().max())
    xh = x.cpu().numpy()
    S = xh != 0
    assert S.any()
    assert np.abs(grad[S] - wl.radius * np.sign(xh[S])).max() <= 1e-6 * scale
    if (~S).any():
        assert np.abs(grad[~S]).max() <= wl.radius + 1e-6 * scale
    del wl
    torch.cuda.empty_cache()


@pytest.mark.parametrize("constraint,csr", [("l1", False), ("l1_penalty", False), ("l2", True),
                                            ("l1", True)])
def test_overlapped_constrained_matches_sequential(gpu_lib, constraint, csr):
    """The overlapped schedule (the next step's sort and Gram beside the
    current pass) forms the same sketches; the gradient is summed in another
    row order, so the iterates agree with the sequential schedule to
    rounding."""
    P = gpu_lib
    if csr:
        wl = W.ridge_csr(rows=1 << 15, d=128, density=8e-3, m=1024, iters=6, radius_factor=0.5)
        M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                     n=wl.n, d=wl.d)
        radius = wl.radius
    else:
        wl = W.lasso_dense(rows=20000, d=64, m=512, iters=6,
                           penalty=40.0 if constraint == "l1_penalty" else None)
        M = P.Matrix(dense=dev(wl.A))
        radius = wl.radius
    runs = {}
    for sched in ("sequential", "overlap"):
        o = P.options(wl.m, seed=wl.sketch_seed, max_iter=6, constraint=constraint,
                      radius=radius, schedule=sched)
        r = P.solve(M, dev(wl.b), o, history=True)
        assert r.report.status == 0 and r.report.qp_unpolished == 0, sched
        runs[sched] = host(r.history)[:, 0, :]
    # the two schedules are two implementations of the same run: the
    # oracle's iterates give the budget of their difference
    if csr:
        c3 = (wl.indptr, wl.indices, wl.data, wl.n, wl.d)
        xs, bud, Aop = oracle_run(None, wl.b, wl.m, 1, wl.sketch_seed, 6, constraint, radius,
                                  csr=c3)
    else:
        xs, bud, Aop = oracle_run(wl.A, wl.b, wl.m, 1, wl.sketch_seed, 6, constraint, radius)
    assert_within_budget(Aop, runs["overlap"], [None] + list(runs["sequential"]), bud)


@pytest.mark.gpu
@pytest.mark.parametrize("d", [32, 128])
def test_overlapped_l1_ball_reports_not_pd_step(gpu_lib, d):
    """The overlapped l1-ball step takes H_t's factor (d = 32) or inverse
    (d = 128) from the side stream; a Hessian sketch that is not positive
    definite (an empty column of A) is reported at the step the sequential
    schedule reports it, and x stays at x^0 = 0."""
    P = gpu_lib
    g = np.random.default_rng(23)
    A = g.standard_normal((4000, d))
    A[:, 7] = 0.0
    b = g.standard_normal(4000)
    reps = {}
    for sched in ("sequential", "overlap"):
        o = P.options(10 * d, seed=5, max_iter=4, constraint="l1", radius=1.0, schedule=sched)
        res = P.solve(P.Matrix(dense=dev(A)), dev(b), o, raise_on_error=False, history=True)
        reps[sched] = (res.report.status, res.report.failed_iter)
        assert bool((res.x == 0).all()), sched
    assert reps["overlap"] == reps["sequential"] == (P.ERR_NOT_PD, 0)


@pytest.mark.gpu
@pytest.mark.parametrize("schedule", ["overlap", "sequential"])
def test_ihs_l2_ragged_batch_matches_oracle(gpu_lib, schedule):
    """A ragged batch through the l2-ball solve: one radius for all
    problems, between the smallest and the largest ||x_OPT||, so some balls
    are active and some inactive, and the problems' shifts (and whether the
    held inverse's series reaches them) differ within each step. Every
    problem's iterates against the oracle's within the rounding budget; each
    problem draws its own sketch stream."""
    P = gpu_lib
    wl = W.batch_ragged(num=4, n_lo=3000, n_hi=8000, d=128, m=1280, iters=8)
    offs = wl.row_offsets
    norms = [np.linalg.norm(O.x_opt(wl.A[offs[p]:offs[p + 1]], wl.b[offs[p]:offs[p + 1]]))
             for p in range(wl.batch)]
    radius = 0.5 * (min(norms) + max(norms))
    o = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l2", radius=radius,
                  schedule=schedule)
    res = P.solve(P.Matrix(dense=dev(wl.A), row_offsets=offs), dev(wl.b), o, history=True)
    assert res.report.status == 0
    hist = host(res.history)
    active = 0
    for p in range(wl.batch):
        Ap, bp = wl.A[offs[p]:offs[p + 1]], wl.b[offs[p]:offs[p + 1]]
        x = np.zeros(wl.d)
        xs, sas, Hs = [x.copy()], [], []
        for t in range(wl.iters):
            SA = OS.sketch_apply_dense(Ap, wl.sketch_seed, t, wl.m, 1, problem=p)
            H = SA.T @ SA
            _, gr, _ = O.gradient(Ap, bp, x)
            x = O.qp_step(H, gr, x, "l2", radius)
            xs.append(x.copy())
            sas.append(SA)
            Hs.append(H)
        active += np.linalg.norm(xs[-1]) > radius * (1 - 1e-9)
        bud = RB.ihs_budget(Ap, bp, sas, Hs, xs, "l2", radius)
        for t in range(wl.iters):
            dx = hist[t, p] - xs[t + 1]
            assert np.linalg.norm(Ap @ dx) <= bud[t][0], (p, t, np.linalg.norm(Ap @ dx),
                                                         bud[t][0])
            assert np.linalg.norm(dx) <= bud[t][1], (p, t)
    assert 0 < active < wl.batch, active


@pytest.mark.gpu
def test_ihs_l2_csr_ragged_batch_matches_oracle(gpu_lib):
    """The l2-ball solve on a ragged batch of CSR problems (rows of one CSR
    matrix split by row_offsets), in the overlapped schedule: one radius for
    all, between the smallest and largest ||x_OPT||; every problem's iterates
    against the oracle's loop on its own rows within the rounding budget."""
    P = gpu_lib
    wl = W.ridge_csr(rows=24000, d=128, density=0.01, m=1024, iters=6)
    offs = np.array([0, 7000, 15000, 24000])
    nb = len(offs) - 1

    def rows(p):
        r0, r1 = int(offs[p]), int(offs[p + 1])
        lo, hi = int(wl.indptr[r0]), int(wl.indptr[r1])
        return (wl.indptr[r0:r1 + 1] - lo, wl.indices[lo:hi], wl.data[lo:hi], r1 - r0, wl.d)

    csrs = [rows(p) for p in range(nb)]
    As = [O.csr_matrix(*c) for c in csrs]
    bs = [wl.b[offs[p]:offs[p + 1]] for p in range(nb)]
    norms = [np.linalg.norm(O.x_opt(As[p], bs[p])) for p in range(nb)]
    radius = 0.5 * (min(norms) + max(norms))
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d, row_offsets=offs)
    o = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, constraint="l2", radius=radius)
    res = P.solve(M, dev(wl.b), o, history=True)
    assert res.report.status == 0
    hist = host(res.history)
    active = 0
    for p in range(nb):
        x = np.zeros(wl.d)
        xs, sas, Hs = [x.copy()], [], []
        for t in range(wl.iters):
            SA = OS.sketch_apply_csr(*csrs[p], wl.sketch_seed, t, wl.m, 1, problem=p)
            H = SA.T @ SA
            _, gr, _ = O.gradient(As[p], bs[p], x)
            x = O.qp_step(H, gr, x, "l2", radius)
            xs.append(x.copy())
            sas.append(SA)
            Hs.append(H)
        active += np.linalg.norm(xs[-1]) > radius * (1 - 1e-9)
        bud = RB.ihs_budget(As[p], bs[p], sas, Hs, xs, "l2", radius)
        for t in range(wl.iters):
            dx = hist[t, p] - xs[t + 1]
            assert np.linalg.norm(As[p] @ dx) <= bud[t][0], (p, t)
            assert np.linalg.norm(dx) <= bud[t][1], (p, t)
    assert 0 < active < nb, active
