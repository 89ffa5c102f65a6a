"""The rounding budget of tests/rounding_budget.py against a second float64
implementation written here: the oracle's own steps with every sum taken in
another order (row blocks of the gradient and sketch rows of the Gram,
reversed) and, for C = R^d, the step applied through an explicit inverse
L^{-T} L^{-1} instead of two triangular solves. The budget must hold for it
at every iterate, and must be exceeded by a run carrying a planted mistake
(the Hessian sketch formed from a float32 copy of S A), so that it tells
rounding from error."""
import numpy as np
import pytest
import scipy.linalg as sla

import rounding_budget as RB
import workloads as W
from oracle import ihs as O
from oracle import sketch as OS


def grad_reordered(A, b, x):
    r = b - A @ x
    g = np.zeros(A.shape[1])
    for rows in np.array_split(np.arange(len(b)), 64)[::-1]:
        g = g + np.asarray(A[rows].T @ r[rows]).ravel()
    return g


def gram_reordered(SA):
    H = np.zeros((SA.shape[1],) * 2)
    for rows in np.array_split(np.arange(SA.shape[0]), 16)[::-1]:
        H = H + SA[rows].T @ SA[rows]
    return H


def step_reordered(H, g, x, constraint, radius):
    if constraint == "none":
        Linv = sla.solve_triangular(np.linalg.cholesky(H), np.eye(len(g)), lower=True)
        return x + (Linv.T @ Linv) @ g
    return O.qp_step(H, g, x, constraint, radius)


def second_run(A, b, sas, x0, constraint, radius, f32_gram=False):
    x = x0.copy()
    out = []
    for SA in sas:
        S = SA.astype(np.float32).astype(np.float64) if f32_gram else SA
        x = step_reordered(gram_reordered(S), grad_reordered(A, b, x), x, constraint, radius)
        out.append(x)
    return out


def budget_case(name):
    if name == "precision":
        wl = W.precision(rows=1 << 13, d=64, m=512, iters=15)
        return wl, wl.A, None, "none", 0.0, 15
    if name == "lasso":
        wl = W.lasso_dense(rows=8000, d=32, m=512, iters=6)
        return wl, wl.A, None, "l1", wl.radius, 6
    if name == "penalty":
        wl = W.lasso_dense(rows=6000, d=24, m=192, penalty=40.0)
        return wl, wl.A, None, "l1_penalty", wl.radius, 8
    wl = W.ridge_csr(rows=1 << 13, d=48, density=3e-2, m=480, iters=6, radius_factor=0.5)
    csr = (wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    return wl, O.csr_matrix(*csr), csr, "l2", wl.radius, 6


@pytest.mark.parametrize("name", ["precision", "lasso", "penalty", "ridge"])
def test_budget_covers_a_reordered_implementation(name):
    wl, A, csr, cons, radius, N = budget_case(name)
    xs, Hs = O.ihs(None if csr else wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=N,
                   constraint=cons, radius=radius, csr=csr, return_hessians=True)
    if csr:
        sas = [OS.sketch_apply_csr(*csr, wl.sketch_seed, t, wl.m) for t in range(N)]
    else:
        sas = [OS.sketch_apply_dense(wl.A, wl.sketch_seed, t, wl.m) for t in range(N)]
    bud = RB.ihs_budget(A, wl.b, sas, Hs, xs, cons, radius)
    other = second_run(A, wl.b, sas, xs[0], cons, radius)
    for t in range(N):
        d = other[t] - xs[t + 1]
        assert np.linalg.norm(A @ d) <= bud[t][0], (t, np.linalg.norm(A @ d), bud[t][0])
        assert np.linalg.norm(d) <= bud[t][1], (t, np.linalg.norm(d), bud[t][1])
    # a planted mistake: the Hessian sketch from float32-rounded S A
    bad = second_run(A, wl.b, sas, xs[0], cons, radius, f32_gram=True)
    assert any(np.linalg.norm(A @ (bad[t] - xs[t + 1])) > bud[t][0] for t in range(N))


def test_budget_shrinks_with_the_error_at_high_conditioning():
    """At kappa(A) = 1e5 the budget follows the IHS error down and stays
    below 1e-3 of it at every step, so it can never hide a step that fails
    to contract."""
    wl, A, _, _, _, N = budget_case("precision")
    xs, Hs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=N, return_hessians=True)
    sas = [OS.sketch_apply_dense(wl.A, wl.sketch_seed, t, wl.m) for t in range(N)]
    bud = RB.ihs_budget(A, wl.b, sas, Hs, xs)
    xo = O.x_opt(wl.A, wl.b)
    for t in range(N):
        assert bud[t][0] < 1e-3 * np.linalg.norm(A @ (xs[t + 1] - xo)), t
    assert bud[-1][0] < 1e-3 * bud[0][0]


def test_float32_accumulated_gram_budget():
    """A Gram accumulated in float32 from S A rounded to float32 (the mixed
    route: both sides round the same float64 S A, so the products agree and
    only the float32 sums differ) stays within the budget with u_g = 2^-24 at
    every iterate; a Gram accumulated at u_g = 2^-16 (planted: every partial
    sum of float32 data rounded to 8 fewer bits) leaves it."""
    wl = W.ols_dense(rows=8000, d=40, m=400, iters=8)
    A, b, N = wl.A, wl.b, 8
    sas = [OS.sketch_apply_dense(A, wl.sketch_seed, t, wl.m, out_dtype="float32")
           for t in range(N)]
    xs, Hs = O.ihs(A, b, wl.m, seed=wl.sketch_seed, iters=N, sketch_dtype="float32",
                   return_hessians=True)
    bud = RB.ihs_budget(A, b, sas, Hs, xs, gram_u=2.0 ** -24)

    def run(round_bits):
        x, out = xs[0].copy(), []
        for SA in sas:
            S32 = SA.astype(np.float32)
            H = np.zeros((A.shape[1],) * 2, dtype=np.float32)
            for k in range(S32.shape[0]):   # sequential float32 accumulation
                H = H + np.outer(S32[k], S32[k])
                if round_bits:
                    m, e = np.frexp(H.astype(np.float64))
                    H = np.ldexp(np.round(m * 2.0 ** round_bits) / 2.0 ** round_bits,
                                 e).astype(np.float32)
            _, g, _ = O.gradient(A, b, x)
            x = O.qp_step(H.astype(np.float64), g, x)
            out.append(x)
        return out

    good = run(0)
    for t in range(N):
        assert np.linalg.norm(A @ (good[t] - xs[t + 1])) <= bud[t][0], t
    bad = run(16)
    assert any(np.linalg.norm(A @ (bad[t] - xs[t + 1])) > bud[t][0] for t in range(N))

