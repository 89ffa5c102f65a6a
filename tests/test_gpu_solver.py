"""GPU parity of the gradient pass, the Gram, the QP step and the IHS loop
against the oracle.

Tolerances follow the arithmetic: a length-k float64 dot product differs
from any other summation order by at most 2 k u sum|terms| (u = 2^-53), so
gradients, Gram entries and objectives are compared componentwise against
those bounds; QP solutions and IHS iterates against a small multiple of the
problem's conditioning times u; the IHS result against x_OPT in the paper's
prediction norm (Def. A.1)."""
import numpy as np
import pytest

import workloads as W
from oracle import ihs as O
from oracle import sketch as OS

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.double().cpu().numpy()


# ------------------------------------------------------------- gradient ----
@pytest.mark.parametrize("n,d", [(5000, 50), (10000, 256), (777, 1024), (1, 3), (300, 511)])
def test_gradient_dense(gpu_lib, n, d):
    P = gpu_lib
    g = np.random.default_rng(n + d)
    A = g.standard_normal((n, d))
    b = g.standard_normal(n)
    x = g.standard_normal(d)
    gg, r, f = P.gradient(P.Matrix(dense=dev(A)), dev(b), dev(x[None, :]), want_r=True)
    r_ref, g_ref, f_ref = O.gradient(A, b, x)
    rb = 2 * d * U * (np.abs(A) @ np.abs(x) + np.abs(b))
    assert np.all(np.abs(host(r) - r_ref) <= rb + 1e-300)
    gb = 4 * (n + d) * U * (np.abs(A).T @ (np.abs(b) + np.abs(A) @ np.abs(x)))
    assert np.all(np.abs(host(gg)[0] - g_ref) <= gb)
    fb = 4 * (n + d) * U * np.sum((np.abs(b) + np.abs(A) @ np.abs(x)) ** 2)
    assert abs(host(f)[0] - f_ref) <= fb


def test_gradient_csr(gpu_lib):
    P = gpu_lib
    wl = W.ridge_csr(rows=30000, d=300, density=0.01)
    A = O.csr_matrix(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    x = np.random.default_rng(1).standard_normal(wl.d)
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d)
    gg, r, f = P.gradient(M, dev(wl.b), dev(x[None, :]), want_r=True)
    r_ref, g_ref, f_ref = O.gradient(A, wl.b, x)
    absA = abs(A)
    scale = absA.T @ (np.abs(wl.b) + absA @ np.abs(x))
    assert np.all(np.abs(host(gg)[0] - g_ref) <= 4 * (wl.n + wl.d) * U * scale)
    assert np.allclose(host(r), r_ref, rtol=0, atol=1e-12)
    assert abs(host(f)[0] - f_ref) <= 1e-12 * f_ref


def csr_rows(wl, r0, r1):
    """Rows r0 .. r1 of a CSR workload as a CSR matrix of their own."""
    lo, hi = int(wl.indptr[r0]), int(wl.indptr[r1])
    return wl.indptr[r0:r1 + 1] - lo, wl.indices[lo:hi], wl.data[lo:hi], r1 - r0


def test_gradient_csr_ragged_batch(gpu_lib):
    """CSR rows split into a ragged batch (an empty problem and a one-row
    problem among them): each problem's gradient and objective against the
    oracle's on its own rows."""
    P = gpu_lib
    wl = W.ridge_csr(rows=12000, d=300, density=0.01)
    offs = np.array([0, 5000, 5000, 5001, 12000])
    X = np.random.default_rng(3).standard_normal((len(offs) - 1, wl.d))
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d, row_offsets=offs)
    gg, _, f = P.gradient(M, dev(wl.b), dev(X))
    for p in range(len(offs) - 1):
        ip, ix, dv, n_p = csr_rows(wl, offs[p], offs[p + 1])
        Ap = O.csr_matrix(ip, ix, dv, n_p, wl.d)
        bp = wl.b[offs[p]:offs[p + 1]]
        _, g_ref, f_ref = O.gradient(Ap, bp, X[p])
        absA = abs(Ap)
        scale = absA.T @ (np.abs(bp) + absA @ np.abs(X[p]))
        assert np.all(np.abs(host(gg)[p] - g_ref) <= 4 * (n_p + wl.d) * U * scale + 1e-300), p
        assert abs(host(f)[p] - f_ref) <= 1e-12 * max(f_ref, 1e-300), p


@pytest.mark.parametrize("schedule", ["overlap", "sequential"])
def test_ihs_csr_ragged_batch(gpu_lib, schedule):
    """IHS on a ragged batch of CSR problems: every problem's iterate after
    each step against the oracle's loop on its own rows, with its own
    sketch stream (problem index p)."""
    P = gpu_lib
    wl = W.ridge_csr(rows=30000, d=80, density=0.02, m=640, iters=6)
    offs = np.array([0, 9000, 21000, 30000])
    M = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                 n=wl.n, d=wl.d, row_offsets=offs)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, schedule=schedule)
    res = P.solve(M, dev(wl.b), opts, history=True)
    assert res.report.status == 0
    hist = host(res.history)
    for p in range(len(offs) - 1):
        ip, ix, dv, n_p = csr_rows(wl, offs[p], offs[p + 1])
        Ap = O.csr_matrix(ip, ix, dv, n_p, wl.d)
        bp = wl.b[offs[p]:offs[p + 1]]
        x = np.zeros(wl.d)
        for t in range(wl.iters):
            SA = OS.sketch_apply_csr(ip, ix, dv, n_p, wl.d, wl.sketch_seed, t, wl.m, 1, problem=p)
            _, gr, _ = O.gradient(Ap, bp, x)
            x = O.qp_step(SA.T @ SA, gr, x)
            assert np.linalg.norm(hist[t, p] - x) <= 1e-11 * np.linalg.norm(x), (p, t)


def test_gradient_ragged_batch(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(2)
    sizes = [1000, 1, 257, 4096]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    A = g.standard_normal((offs[-1], 64))
    b = g.standard_normal(offs[-1])
    X = g.standard_normal((len(sizes), 64))
    gg, _, f = P.gradient(P.Matrix(dense=dev(A), row_offsets=offs), dev(b), dev(X))
    for p in range(len(sizes)):
        Ap, bp = A[offs[p]:offs[p + 1]], b[offs[p]:offs[p + 1]]
        _, g_ref, f_ref = O.gradient(Ap, bp, X[p])
        assert np.allclose(host(gg)[p], g_ref, rtol=1e-11, atol=1e-10)
        assert np.isclose(host(f)[p], f_ref, rtol=1e-12)


# ----------------------------------------------------------------- Gram ----
@pytest.mark.parametrize("m,d,batch", [(500, 50, 1), (4096, 256, 1), (640, 64, 3),
                                       (100, 33, 1), (8192, 1024, 1), (3, 5, 2)])
def test_gram_f64(gpu_lib, m, d, batch):
    P = gpu_lib
    g = np.random.default_rng(m + d)
    SA = g.standard_normal((batch * m, d))
    H = host(P.gram(dev(SA), m, batch=batch))
    for p in range(batch):
        S = SA[p * m:(p + 1) * m]
        ref = O.gram(S)
        bound = 2 * m * U * (np.abs(S).T @ np.abs(S))
        assert np.all(np.abs(H[p] - ref) <= bound), p
        assert np.array_equal(H[p], H[p].T)


@pytest.mark.parametrize("in_dt,acc", [("float32", "float64"), ("float32", "float32"),
                                       ("bfloat16", "float32")])
def test_gram_mixed(gpu_lib, in_dt, acc):
    import torch
    P = gpu_lib
    g = np.random.default_rng(3)
    m, d = 2048, 160
    SA64 = g.standard_normal((m, d))
    SA_in = OS.round_output(SA64, in_dt)
    # SA_in holds values exactly representable in the input type, so the cast is exact
    t = dev(np.asarray(SA_in, dtype=np.float64)).to(
        torch.float32 if in_dt == "float32" else torch.bfloat16)
    assert np.array_equal(host(t), np.asarray(SA_in, dtype=np.float64))
    H = host(P.gram(t, m, in_dtype=in_dt, acc_dtype=acc))[0]
    S = np.asarray(SA_in, dtype=np.float64)
    ref = S.T @ S
    u_acc = 2.0 ** -24 if acc == "float32" else U
    bound = 2 * m * u_acc * (np.abs(S).T @ np.abs(S))
    assert np.all(np.abs(H - ref) <= bound)


# ------------------------------------------------------------------- QP ----
def spd(d, g, cond):
    Q, _ = np.linalg.qr(g.standard_normal((d, d)))
    return Q @ np.diag(np.geomspace(1.0, cond, d)) @ Q.T


@pytest.mark.parametrize("d,batch", [(50, 1), (64, 4), (256, 1), (512, 1), (130, 2), (1, 1),
                                     (1024, 1), (2, 1), (63, 2), (65, 1), (88, 1), (89, 1),
                                     (127, 1), (128, 1), (129, 3), (577, 1)])
def test_qp_unconstrained(gpu_lib, d, batch):
    P = gpu_lib
    g = np.random.default_rng(d)
    Hs = np.stack([spd(d, g, 1e3) for _ in range(batch)])
    gs = g.standard_normal((batch, d))
    xs = g.standard_normal((batch, d))
    out = host(P.qp_step(dev(Hs), dev(gs), dev(xs)))
    for p in range(batch):
        ref = O.qp_step(Hs[p], gs[p], xs[p])
        dx, dref = out[p] - xs[p], ref - xs[p]
        assert np.linalg.norm(dx - dref) <= 1e-12 * 1e3 * np.linalg.norm(dref) * max(1, d / 64)


@pytest.mark.parametrize("d,bad,value", [(200, 150, -1.0), (40, 10, -1.0), (64, 63, 0.0),
                                         (100, 70, float("nan"))])
def test_qp_not_positive_definite(gpu_lib, d, bad, value):
    """A negative, zero or NaN pivot, in the first diagonal block, its last
    column or a later block, is reported as not positive definite."""
    P = gpu_lib
    H = np.eye(d)
    H[bad, bad] = value
    with pytest.raises(P.IHSError) as e:
        P.qp_step(dev(H[None]), dev(np.ones((1, d))), dev(np.zeros((1, d))))
    assert e.value.code == P.ERR_NOT_PD


# ------------------------------------------------------------------ IHS ----
def test_ihs_unconstrained_iterates_match_oracle(gpu_lib):
    P = gpu_lib
    wl = W.ols_dense(rows=20000, d=50, m=500, iters=10)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters)
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0 and res.report.iters == wl.iters
    xs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=wl.iters)
    hist = host(res.history)[:, 0, :]
    for t in range(wl.iters):
        assert np.linalg.norm(hist[t] - xs[t + 1]) <= 1e-11 * np.linalg.norm(xs[t + 1]), t
    xo = O.x_opt(wl.A, wl.b)
    errs = [O.error_A(wl.A, hist[t], xo) for t in range(wl.iters)]
    assert errs[-1] < errs[0] * 0.6 ** 9
    r_ref, _, f_ref = O.gradient(wl.A, wl.b, xs[wl.iters - 1])
    assert abs(res.report.objective - f_ref) <= 1e-11 * f_ref


@pytest.mark.parametrize("gin,gacc", [("float64", "float64"), ("float32", "float64"),
                                      ("float32", "float32"), ("bfloat16", "float32")])
def test_ihs_f32_data_and_mixed_gram(gpu_lib, gin, gacc):
    """float32 data with each Gram route, every iterate against the oracle's
    run with S A rounded the same way (the Gram of the rounded inputs formed
    in float64) within the rounding budget: the GPU's Gram rounds at u for
    a float64 accumulation (the products of rounded inputs are exact), at
    2^-24 for a float32 one."""
    P = gpu_lib
    import rounding_budget as RB
    wl = W.ols_dense(rows=8000, d=40, m=400, iters=8)
    A32 = wl.A.astype(np.float32)
    A64 = A32.astype(np.float64)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, gram_in=gin, gram_acc=gacc)
    res = P.solve(P.Matrix(dense=dev(A32)), dev(wl.b), opts, history=True)
    hist = host(res.history)[:, 0, :]
    xs, Hs = O.ihs(A64, wl.b, wl.m, seed=wl.sketch_seed, iters=wl.iters, sketch_dtype=gin,
                   return_hessians=True)
    sas = [OS.sketch_apply_dense(A64, wl.sketch_seed, t, wl.m, out_dtype=gin)
           for t in range(wl.iters)]
    gram_u = 2.0 ** -24 if gacc == "float32" else 2.0 ** -53
    bud = RB.ihs_budget(A64, wl.b, sas, Hs, xs, gram_u=gram_u)
    for t in range(wl.iters):
        dx = hist[t] - xs[t + 1]
        assert np.linalg.norm(A64 @ dx) <= bud[t][0], (gin, gacc, t, np.linalg.norm(A64 @ dx),
                                                      bud[t][0])
        assert np.linalg.norm(dx) <= bud[t][1], (gin, gacc, t)
    # and the method converges at its rate (about 0.37 per step at m = 10 d)
    xo = O.x_opt(A64, wl.b)
    assert O.error_A(A64, hist[-1], xo) < 3e-3


def test_ihs_ragged_batch(gpu_lib):
    P = gpu_lib
    wl = W.batch_ragged(num=6, n_lo=2000, n_hi=9000, d=64, iters=12)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters)
    res = P.solve(P.Matrix(dense=dev(wl.A), row_offsets=wl.row_offsets), dev(wl.b), opts)
    X = host(res.x)
    for p in range(wl.batch):
        r0, r1 = wl.row_offsets[p], wl.row_offsets[p + 1]
        Ap = wl.A[r0:r1]
        # the oracle draws problem p's sketch with problem index p
        x = np.zeros(64)
        for t in range(wl.iters):
            SA = OS.sketch_apply_dense(Ap, wl.sketch_seed, t, wl.m, 1, problem=p)
            _, gr, _ = O.gradient(Ap, wl.b[r0:r1], x)
            x = O.qp_step(SA.T @ SA, gr, x)
        assert np.linalg.norm(X[p] - x) <= 1e-11 * np.linalg.norm(x), p
        assert O.error_A(Ap, X[p], O.x_opt(Ap, wl.b[r0:r1])) < 1e-4


def test_ihs_rank_deficient_reports_not_pd(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(9)
    A = g.standard_normal((2000, 20))
    A[:, 7] = 0.0                           # empty column: H exactly singular
    b = g.standard_normal(2000)
    opts = P.options(200, seed=1, max_iter=3)
    res = P.solve(P.Matrix(dense=dev(A)), dev(b), opts, raise_on_error=False)
    assert res.report.status == P.ERR_NOT_PD
    assert res.report.failed_iter == 0


def test_ihs_nonfinite_objective_detected(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(10)
    A = g.standard_normal((3000, 16))
    b = g.standard_normal(3000)
    b[123] = np.nan
    res = P.solve(P.Matrix(dense=dev(A)), dev(b), P.options(160, max_iter=2),
                  raise_on_error=False)
    assert res.report.status == P.ERR_NONFINITE


def test_ihs_deterministic(gpu_lib):
    P = gpu_lib
    wl = W.lasso_dense(rows=30000, d=128, m=1024)
    opts = P.options(1024, seed=3, max_iter=4)
    M = P.Matrix(dense=dev(wl.A))
    a = P.solve(M, dev(wl.b), opts).x
    b = P.solve(M, dev(wl.b), opts).x
    assert bool((a == b).all())


@pytest.mark.parametrize("shape", [(30000, 64, 640, 1), (20000, 256, 2048, 1), (9000, 40, 400, 3),
                                   (12000, 150, 1500, 2), (40000, 578, 5000, 1)])
def test_overlap_schedule_matches_sequential(gpu_lib, shape):
    P = gpu_lib
    n, d, m, batch = shape
    g = np.random.default_rng(n + d)
    A = g.standard_normal((n, d))
    b = g.standard_normal(n)
    offs = None if batch == 1 else np.linspace(0, n, batch + 1).astype(np.int64)
    M = P.Matrix(dense=dev(A), row_offsets=offs)
    out = {}
    for sched in ("overlap", "overlap2", "sequential"):
        opts = P.options(m, seed=17, iter0=5, max_iter=7, schedule=sched)
        r = P.solve(M, dev(b), opts, history=True, factors=True)
        out[sched] = (host(r.x), host(r.history), host(r.factors), r.report)
    s = out["sequential"]
    for sched in ("overlap", "overlap2"):
        a = out[sched]
        # same sketches, so the same factors bit for bit; the gradient is summed
        # in another row order (and wide problems apply an explicit inverse),
        # so iterates agree to rounding
        assert np.array_equal(a[2], s[2]), sched
        for t in range(7):
            assert np.allclose(a[1][t], s[1][t], rtol=1e-12,
                               atol=1e-14 * np.abs(s[1][t]).max()), (sched, t)
        assert a[3].status == s[3].status == 0
        assert abs(a[3].objective - s[3].objective) <= 1e-12 * s[3].objective


def test_overlap_reports_not_pd_step(gpu_lib):
    P = gpu_lib
    g = np.random.default_rng(21)
    A = g.standard_normal((4000, 32))
    A[:, 5] = 0.0
    res = P.solve(P.Matrix(dense=dev(A)), dev(g.standard_normal(4000)),
                  P.options(320, max_iter=4), raise_on_error=False, history=True)
    assert res.report.status == P.ERR_NOT_PD and res.report.failed_iter == 0
    assert bool((res.x == 0).all())


def test_largest_sketch_overlapped_iterates_match_oracle(gpu_lib):
    """m = 16384, the largest sketch the library takes per problem, on the
    overlapped schedule the benchmark times for its larger-sketch variants:
    every iterate matches the oracle's, and the error contracts faster per
    step than at m = 8 d."""
    P = gpu_lib
    wl = W.ols_dense(rows=60000, d=96, m=16384, iters=6)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=wl.iters, schedule="overlap")
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0 and res.report.iters == wl.iters
    xs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=wl.iters)
    hist = host(res.history)[:, 0, :]
    xo = O.x_opt(wl.A, wl.b)
    for t in range(wl.iters):
        assert np.linalg.norm(hist[t] - xs[t + 1]) <= 1e-11 * np.linalg.norm(xs[t + 1]), t
    errs = [O.error_A(wl.A, hist[t], xo) for t in range(wl.iters)]
    assert errs[3] < 0.2 ** 4


# ---------------------------------- one fixed sketch + conjugate gradients ----
@pytest.mark.parametrize("n,d,m,iters", [(20000, 50, 400, 12), (30000, 120, 960, 10),
                                         (5000, 7, 56, 7)])
def test_fixed_sketch_cg_iterates_match_oracle(gpu_lib, n, d, m, iters):
    """Dense A through both preconditioner paths (triangular solves below
    d = 89, the explicit inverse above): every iterate matches the oracle's,
    and the A-norm error falls below IHS's after the same number of passes."""
    P = gpu_lib
    wl = W.ols_dense(rows=n, d=d, m=m, iters=iters)
    opts = P.options(wl.m, seed=wl.sketch_seed, iter0=3, max_iter=iters,
                     method="fixed_sketch_cg")
    res = P.solve(P.Matrix(dense=dev(wl.A)), dev(wl.b), opts, history=True)
    assert res.report.status == 0 and res.report.iters == iters
    xs = O.fixed_sketch_cg(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iter0=3, iters=iters)
    hist = host(res.history)[:, 0, :]
    xo = O.x_opt(wl.A, wl.b)
    for t in range(iters):
        scale = max(np.linalg.norm(xs[t + 1]), 1e-300)
        assert np.linalg.norm(hist[t] - xs[t + 1]) <= 1e-10 * scale, t
    r0 = wl.b  # the objective is reported at x^0 = 0
    assert abs(res.report.objective - 0.5 * r0 @ r0) <= 1e-12 * (0.5 * r0 @ r0)
    if d < n // 100:
        ih = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iter0=3, iters=iters)
        assert O.error_A(wl.A, hist[-1], xo) < O.error_A(wl.A, ih[-1], xo)


def test_fixed_sketch_cg_csr_and_ragged_batch(gpu_lib):
    P = gpu_lib
    # CSR
    wl = W.ridge_csr(rows=40000, d=64, density=0.05, m=512, iters=8)
    import torch
    M = P.Matrix(row_ptr=torch.from_numpy(wl.indptr).cuda(),
                 col_idx=torch.from_numpy(wl.indices).cuda(),
                 values=torch.from_numpy(wl.data).cuda(), n=wl.n, d=wl.d)
    opts = P.options(wl.m, seed=wl.sketch_seed, max_iter=8, method="fixed_sketch_cg")
    res = P.solve(M, dev(wl.b), opts, history=True)
    assert res.report.status == 0
    csr = (wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    xs = O.fixed_sketch_cg(None, wl.b, wl.m, seed=wl.sketch_seed, iters=8, csr=csr)
    hist = host(res.history)[:, 0, :]
    for t in range(8):
        assert np.linalg.norm(hist[t] - xs[t + 1]) <= 1e-10 * np.linalg.norm(xs[t + 1]), t
    # ragged batch: problem p draws its sketch with problem index p
    wb = W.batch_ragged(num=5, n_lo=1500, n_hi=7000, d=32, iters=6)
    opts = P.options(wb.m, seed=wb.sketch_seed, max_iter=6, method="fixed_sketch_cg")
    res = P.solve(P.Matrix(dense=dev(wb.A), row_offsets=wb.row_offsets), dev(wb.b), opts)
    X = host(res.x)
    for p in range(wb.batch):
        r0, r1 = wb.row_offsets[p], wb.row_offsets[p + 1]
        ref = O.fixed_sketch_cg(wb.A[r0:r1], wb.b[r0:r1], wb.m, seed=wb.sketch_seed, iters=6,
                                problem=p)[-1]
        assert np.linalg.norm(X[p] - ref) <= 1e-10 * np.linalg.norm(ref), p


def test_fixed_sketch_cg_rank_deficient_reports_not_pd(gpu_lib):
    """An empty column makes H_0 exactly singular: the factorisation reports
    it and x keeps its start."""
    P = gpu_lib
    g = np.random.default_rng(5)
    A = g.standard_normal((3000, 6))
    A[:, 4] = 0.0
    opts = P.options(60, seed=2, max_iter=4, method="fixed_sketch_cg")
    res = P.solve(P.Matrix(dense=dev(A)), dev(g.standard_normal(3000)), opts,
                  raise_on_error=False)
    assert res.report.status == P.ERR_NOT_PD
    assert np.array_equal(host(res.x), np.zeros((1, 6)))
