"""Pins for the oracle's Gram, gradient, QP solvers, IHS loop, x_OPT, error
metric and derivatives: math.fsum, closed forms, hand-solved projections, KKT
conditions, brute-force enumeration, an independent constrained solver, the
exact IHS error recurrence, Thm 2.2's geometric decay and finite differences."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import optimize

from oracle import ihs as O
from oracle.sketch import sketch_apply_dense, sketch_hash
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


# ------------------------------------------------------------------ Gram ----
def test_gram_fsum_bound_and_symmetry():
    g = np.random.default_rng(0)
    SA = g.standard_normal((300, 7))
    H = O.gram(SA)
    m = SA.shape[0]
    for j in range(7):
        for k in range(7):
            terms = SA[:, j] * SA[:, k]
            exact = math.fsum(terms)
            assert abs(H[j, k] - exact) <= 2 * m * U * np.abs(terms).sum()
    assert np.array_equal(H, H.T)
    assert np.linalg.eigvalsh(H).min() > 0


def test_gram_mixed_rounds_inputs_once():
    g = np.random.default_rng(1)
    SA = g.standard_normal((64, 5))
    H32 = O.gram_mixed(SA, "float32")
    SA32 = SA.astype(np.float32).astype(np.float64)
    assert np.allclose(H32, SA32.T @ SA32, rtol=1e-15, atol=1e-13)
    Hb = O.gram_mixed(SA, "bfloat16")
    assert np.all(np.abs(Hb - O.gram(SA)) <= 3 * 2.0 ** -8 * (np.abs(SA).T @ np.abs(SA)))


# -------------------------------------------------------------- gradient ----
def test_gradient_at_zero_is_Atb_and_fsum():
    g = np.random.default_rng(2)
    A = g.standard_normal((200, 4))
    b = g.standard_normal(200)
    r, gr, f = O.gradient(A, b, np.zeros(4))
    assert np.array_equal(r, b)
    for j in range(4):
        terms = A[:, j] * b
        assert abs(gr[j] - math.fsum(terms)) <= 200 * U * np.abs(terms).sum()
    assert abs(f - 0.5 * math.fsum(b * b)) <= 200 * U * (b * b).sum()


def test_gradient_is_minus_derivative_of_objective():
    g = np.random.default_rng(3)
    A = g.standard_normal((50, 6))
    b = g.standard_normal(50)
    x = g.standard_normal(6)
    _, gr, _ = O.gradient(A, b, x)
    f = lambda z: 0.5 * np.sum((A @ z - b) ** 2)
    for _ in range(5):
        v = g.standard_normal(6)
        h = 1e-5
        fd = (f(x + h * v) - f(x - h * v)) / (2 * h)
        assert abs(fd + gr @ v) < 1e-7 * (1 + abs(fd))


def test_gradient_vanishes_at_x_opt_within_bound():
    g = np.random.default_rng(4)
    A = g.standard_normal((500, 8))
    b = A @ g.standard_normal(8) + 0.1 * g.standard_normal(500)
    x = O.x_opt(A, b)
    _, gr, _ = O.gradient(A, b, x)
    bound = 4 * 500 * U * (np.abs(A).T @ (np.abs(b) + np.abs(A) @ np.abs(x)))
    assert np.all(np.abs(gr) <= bound)


def test_csr_gradient_matches_dense():
    wl = W.ridge_csr(rows=3000, d=40, density=0.05)
    A = O.csr_matrix(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    D = W.csr_to_dense(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    x = np.random.default_rng(5).standard_normal(wl.d)
    r1, g1, f1 = O.gradient(A, wl.b, x)
    r2, g2, f2 = O.gradient(D, wl.b, x)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-10)
    assert np.allclose(r1, r2, rtol=1e-13, atol=1e-13) and math.isclose(f1, f2, rel_tol=1e-12)


# ------------------------------------------------------------------- QP ----
def random_spd(d, g, cond=10.0):
    Q, _ = np.linalg.qr(g.standard_normal((d, d)))
    return Q @ np.diag(np.geomspace(1.0, cond, d)) @ Q.T


def test_unconstrained_step_solves_normal_system():
    g = np.random.default_rng(6)
    H = random_spd(12, g, 1e4)
    gr = g.standard_normal(12)
    x0 = g.standard_normal(12)
    x1 = O.qp_step(H, gr, x0)
    assert np.linalg.norm(H @ (x1 - x0) - gr) <= 50 * 12 * U * np.linalg.norm(H, 2) * np.linalg.norm(x1 - x0)


def test_not_positive_definite_is_reported():
    H = np.diag([1.0, 0.0, 2.0])
    with pytest.raises(O.NotPositiveDefinite):
        O.qp_step(H, np.ones(3), np.zeros(3))


def test_l1_projection_golden_cases():
    with open(os.path.join(GOLDEN, "l1_projection_cases.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        assert np.allclose(O.project_l1_ball(np.array(c["v"]), c["tau"]), c["x"],
                           rtol=0, atol=1e-15), c


def test_l1_projection_variational_inequality():
    g = np.random.default_rng(7)
    for _ in range(50):
        v = g.standard_normal(9) * 3
        tau = g.uniform(0.1, 5)
        p = O.project_l1_ball(v, tau)
        assert np.abs(p).sum() <= tau * (1 + 1e-12)
        for _ in range(20):
            z = O.project_l1_ball(g.standard_normal(9) * 3, tau)
            assert (v - p) @ (z - p) <= 1e-10


def brute_force_l1(H, c, tau):
    """Exact minimiser over the ball by enumerating every face: interior
    (unconstrained) plus each support/sign pattern on the surface."""
    d = len(c)
    best, best_x = np.inf, None
    obj = lambda x: 0.5 * x @ H @ x - c @ x
    x_unc = np.linalg.solve(H, c)
    if np.abs(x_unc).sum() <= tau:
        return x_unc
    for pattern in itertools.product((-1, 0, 1), repeat=d):
        sig = np.array(pattern, dtype=float)
        S = np.nonzero(sig)[0]
        if len(S) == 0:
            continue
        K = np.zeros((len(S) + 1, len(S) + 1))
        K[:-1, :-1] = H[np.ix_(S, S)]
        K[:-1, -1] = sig[S]
        K[-1, :-1] = sig[S]
        rhs = np.concatenate([c[S], [tau]])
        sol = np.linalg.solve(K, rhs)
        xs = sol[:-1]
        if np.any(np.sign(xs) != sig[S]):
            continue
        x = np.zeros(d)
        x[S] = xs
        if obj(x) < best:
            best, best_x = obj(x), x
    return best_x


def test_l1_qp_matches_brute_force():
    g = np.random.default_rng(8)
    for trial in range(12):
        d = 5
        H = random_spd(d, g, 20.0)
        c = g.standard_normal(d) * 3
        x_unc = np.linalg.solve(H, c)
        tau = np.abs(x_unc).sum() * g.uniform(0.2, 1.2)
        x = O.qp_l1(H, c, tau)
        assert np.allclose(x, brute_force_l1(H, c, tau), rtol=1e-10, atol=1e-12), trial


def test_l1_qp_kkt_larger():
    g = np.random.default_rng(9)
    d = 40
    H = random_spd(d, g, 9.0)
    c = g.standard_normal(d) * 2
    tau = 0.3 * np.abs(np.linalg.solve(H, c)).sum()
    x = O.qp_l1(H, c, tau)
    assert abs(np.abs(x).sum() - tau) < 1e-12 * tau
    grad = c - H @ x
    S = x != 0
    mu = np.mean(grad[S] * np.sign(x[S]))
    assert mu > 0
    assert np.allclose(grad[S], mu * np.sign(x[S]), atol=1e-11)
    assert np.all(np.abs(grad[~S]) <= mu + 1e-11)


def test_l2_qp_identity_closed_form_and_inactive():
    g = np.random.default_rng(10)
    c = g.standard_normal(6)
    r = 0.5 * np.linalg.norm(c)
    assert np.allclose(O.qp_l2(np.eye(6), c, r), c * r / np.linalg.norm(c), atol=1e-14)
    assert np.allclose(O.qp_l2(np.eye(6), c, 10 * np.linalg.norm(c)), c, atol=1e-15)
    H = random_spd(6, g, 50)
    big = 10 * np.linalg.norm(np.linalg.solve(H, c))
    assert np.allclose(O.qp_l2(H, c, big), np.linalg.solve(H, c), rtol=1e-13)


def test_l2_qp_kkt_and_scipy():
    g = np.random.default_rng(11)
    d = 6
    H = random_spd(d, g, 100)
    c = g.standard_normal(d)
    r = 0.3 * np.linalg.norm(np.linalg.solve(H, c))
    x = O.qp_l2(H, c, r)
    assert abs(np.linalg.norm(x) - r) < 1e-12 * r
    # KKT: c - H x = mu x with mu >= 0
    mu = (c - H @ x) @ x / (x @ x)
    assert mu > 0 and np.allclose(c - H @ x, mu * x, atol=1e-11)
    res = optimize.minimize(lambda z: 0.5 * z @ H @ z - c @ z, np.zeros(d),
                            jac=lambda z: H @ z - c, method="SLSQP",
                            constraints=[{"type": "ineq", "fun": lambda z: r * r - z @ z,
                                          "jac": lambda z: -2 * z}],
                            options={"ftol": 1e-14, "maxiter": 500})
    assert np.allclose(x, res.x, atol=1e-6)


# --------------------------------------------------------------- x_OPT ----
def test_x_opt_lstsq_matches_qr():
    g = np.random.default_rng(12)
    A = g.standard_normal((400, 10))
    b = g.standard_normal(400)
    Q, R = np.linalg.qr(A)
    assert np.allclose(O.x_opt(A, b), sla.solve_triangular(R, Q.T @ b), rtol=1e-12)


def test_precision_structural_x_opt():
    """x_OPT for A = G diag(sigma) V equals V^T diag(1/sigma) argmin_y ||G y - b||
    up to the rounding of the stored product (A-norm)."""
    wl = W.precision(rows=4096, d=32, m=256, kappa=1e5, keep_factors=True)
    A, b = wl.A, wl.b
    G = wl.meta["G"].astype(np.float64)
    y = np.linalg.lstsq(G, b, rcond=None)[0]
    x_struct = wl.meta["V"].T @ (y / wl.meta["sigma"])
    x = O.x_opt(A, b)
    assert O.error_A(A, x_struct, x) < 1e-12


def test_error_metric_is_prediction_norm_ratio():
    g = np.random.default_rng(13)
    A = g.standard_normal((30, 3))
    x, xr = g.standard_normal(3), g.standard_normal(3)
    n = 30
    anorm = lambda v: np.linalg.norm(A @ v) / math.sqrt(n)
    assert math.isclose(O.error_A(A, x, xr), anorm(x - xr) / anorm(xr), rel_tol=1e-14)


# ---------------------------------------------------------------- IHS ----
def test_ihs_exact_error_recurrence():
    g = np.random.default_rng(14)
    n, d, m = 2000, 10, 80
    A = g.standard_normal((n, d))
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    xo = O.x_opt(A, b)
    xs, Hs = O.ihs(A, b, m, seed=5, iters=6, return_hessians=True)
    e = -xo
    for t, H in enumerate(Hs):
        e = e - np.linalg.solve(H, A.T @ (A @ e))
        assert np.allclose(xs[t + 1] - xo, e, rtol=1e-8, atol=1e-12 * np.linalg.norm(xo))


def test_ihs_collision_free_sketch_converges_in_one_step():
    g = np.random.default_rng(15)
    n, d, m = 14, 3, 1 << 22
    A = g.standard_normal((n, d))
    b = g.standard_normal(n)
    bucket, _ = sketch_hash(3, 0, n, m, 1)
    assert len(np.unique(bucket)) == n
    xs = O.ihs(A, b, m, seed=3, iters=1)
    assert O.error_A(A, xs[1], O.x_opt(A, b)) < 1e-13


def test_ihs_geometric_decay_thm22():
    wl = W.ols_dense(rows=20000, d=50, m=500)
    xo = O.x_opt(wl.A, wl.b)
    xs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=10)
    errs = [O.error_A(wl.A, x, xo) for x in xs[1:]]
    ratios = np.array(errs[1:8]) / np.array(errs[:7])
    assert np.all(ratios < 0.6)
    assert errs[-1] < errs[0] * 0.6 ** 9


def test_ihs_sjlt_and_countsketch_converge_l1():
    wl = W.lasso_dense(rows=6000, d=24, m=192)
    xo = O.x_opt(wl.A, wl.b, "l1", wl.radius)
    # KKT of the full problem at x_OPT
    AtA, Atb = wl.A.T @ wl.A, wl.A.T @ wl.b
    grad = Atb - AtA @ xo
    S = xo != 0
    mu = np.mean(grad[S] * np.sign(xo[S]))
    assert mu > 0 and np.all(np.abs(grad[~S]) <= mu * (1 + 1e-8))
    for kind, s in (("countsketch", 1), ("sjlt", 4)):
        xs = O.ihs(wl.A, wl.b, wl.m, s=s, seed=wl.sketch_seed, iters=14,
                   constraint="l1", radius=wl.radius)
        assert O.error_A(wl.A, xs[-1], xo) < 1e-8, kind


def test_ihs_l2_csr_converges():
    wl = W.ridge_csr(rows=20000, d=32, density=0.03, m=256, radius_factor=0.5)
    A = O.csr_matrix(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    xo = O.x_opt(A, wl.b, "l2", wl.radius)
    assert abs(np.linalg.norm(xo) - wl.radius) < 1e-10 * wl.radius
    xs = O.ihs(None, wl.b, wl.m, seed=wl.sketch_seed, iters=12, constraint="l2",
               radius=wl.radius, csr=(wl.indptr, wl.indices, wl.data, wl.n, wl.d))
    assert O.error_A(A, xs[-1], xo) < 1e-8


# ---------------------------------------------------------- derivatives ----
def test_closed_form_gradients_match_finite_differences():
    g = np.random.default_rng(16)
    n, d = 300, 5
    A = g.standard_normal((n, d))
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    y = g.standard_normal(d)
    L0, dLdb, dLdA = O.loss_and_grads_closed_form(A, b, y)
    Lf = lambda A_, b_: float(np.sum((np.linalg.lstsq(A_, b_, rcond=None)[0] - y) ** 2))
    h = 1e-6
    for _ in range(4):
        Eb = g.standard_normal(n)
        fd = (Lf(A, b + h * Eb) - Lf(A, b - h * Eb)) / (2 * h)
        assert abs(fd - dLdb @ Eb) < 1e-6 * (1 + abs(fd))
        EA = g.standard_normal((n, d))
        fd = (Lf(A + h * EA, b) - Lf(A - h * EA, b)) / (2 * h)
        assert abs(fd - np.sum(dLdA * EA)) < 1e-6 * (1 + abs(fd))


def test_adjoint_ihs_converges_to_closed_form():
    g = np.random.default_rng(17)
    n, d, m = 4000, 8, 80
    A = g.standard_normal((n, d))
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    y = g.standard_normal(d)
    xs, Hs = O.ihs(A, b, m, seed=9, iters=20, return_hessians=True)
    _, dLdb, dLdA = O.loss_and_grads_closed_form(A, b, y)
    lam = O.adjoint_ihs(A, Hs, 2 * (xs[-1] - y))
    gb, gA = O.grads_from_lambda(A, b, xs[-1], lam)
    assert np.allclose(gb, dLdb, rtol=1e-8, atol=1e-10)
    assert np.allclose(gA, dLdA, rtol=1e-8, atol=1e-10)


# ----------------------------------------------- precision feasibility ----
def test_precision_variants_on_scaled_ill_conditioned_problem():
    """A Gram from float32-rounded SA converges like float64 at kappa = 1e5, while a
    bfloat16-rounded SA stalls: the input rounding perturbs H by about
    kappa * u_in relative to its smallest eigenvalue."""
    wl = W.precision(rows=16384, d=32, m=256, kappa=1e5)
    xo = O.x_opt(wl.A, wl.b)
    e = {}
    for dt in ("float64", "float32", "bfloat16"):
        xs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=30, sketch_dtype=dt)
        e[dt] = O.error_A(wl.A, xs[-1], xo)
    assert e["float64"] < 1e-9 and e["float32"] < 1e-9
    assert e["bfloat16"] > 1e-4


# ------------------------------------------------- penalised LASSO step ----
def brute_force_l1_penalty(H, c, lam):
    """Exact minimiser of 1/2 x^T H x - c^T x + lam ||x||_1 by enumerating every
    support/sign pattern: on a pattern the objective is a smooth quadratic whose
    stationary point solves H_SS x_S = c_S - lam sigma_S; among the patterns
    whose solution keeps its signs, the smallest objective is the minimum."""
    d = len(c)
    obj = lambda x: 0.5 * x @ H @ x - c @ x + lam * np.abs(x).sum()
    best_x = np.zeros(d)
    best = obj(best_x)
    for pattern in itertools.product((-1, 0, 1), repeat=d):
        sig = np.array(pattern, dtype=float)
        S = np.nonzero(sig)[0]
        if len(S) == 0:
            continue
        xs = np.linalg.solve(H[np.ix_(S, S)], c[S] - lam * sig[S])
        if np.any(np.sign(xs) != sig[S]):
            continue
        x = np.zeros(d)
        x[S] = xs
        if obj(x) < best:
            best, best_x = obj(x), x
    return best_x


def test_l1_penalty_closed_forms():
    g = np.random.default_rng(21)
    c = g.standard_normal(9) * 2
    lam = 0.7
    # H = I: the soft threshold of c; H diagonal: its per-coordinate scaling
    assert np.allclose(O.qp_l1_penalty(np.eye(9), c, lam), O.soft_threshold(c, lam),
                       rtol=1e-14, atol=0)
    h = g.uniform(0.5, 3.0, 9)
    assert np.allclose(O.qp_l1_penalty(np.diag(h), c, lam),
                       np.sign(c) * np.maximum(np.abs(c) - lam, 0) / h, rtol=1e-14, atol=0)
    # hand-checked soft threshold values
    assert np.array_equal(O.soft_threshold(np.array([3.0, -2.5, 0.4, -0.1, 1.0]), 1.0),
                          np.array([2.0, -1.5, 0.0, -0.0, 0.0]))
    # a weight at or above max |c| gives 0
    H = random_spd(9, g, 10.0)
    assert np.array_equal(O.qp_l1_penalty(H, c, np.abs(c).max()), np.zeros(9))


def test_l1_penalty_qp_matches_brute_force():
    g = np.random.default_rng(22)
    for trial in range(12):
        d = 5
        H = random_spd(d, g, 20.0)
        c = g.standard_normal(d) * 3
        lam = g.uniform(0.05, 0.8) * np.abs(c).max()
        x = O.qp_l1_penalty(H, c, lam)
        assert np.allclose(x, brute_force_l1_penalty(H, c, lam), rtol=1e-10, atol=1e-12), trial


def test_l1_penalty_kkt_larger_and_zero_weight():
    g = np.random.default_rng(23)
    d = 40
    H = random_spd(d, g, 9.0)
    c = g.standard_normal(d) * 2
    lam = 0.5
    x = O.qp_l1_penalty(H, c, lam)
    grad = c - H @ x
    S = x != 0
    assert 0 < S.sum() < d
    assert np.allclose(grad[S], lam * np.sign(x[S]), atol=1e-11)
    assert np.all(np.abs(grad[~S]) <= lam + 1e-11)
    # lambda = 0 is the unconstrained minimiser
    d0 = 8
    H0 = random_spd(d0, g, 5.0)
    c0 = g.standard_normal(d0)
    assert np.allclose(O.qp_l1_penalty(H0, c0, 0.0), np.linalg.solve(H0, c0), rtol=1e-12)


def test_ihs_l1_penalty_converges():
    wl = W.lasso_dense(rows=6000, d=24, m=192, penalty=40.0)
    xo = O.x_opt(wl.A, wl.b, "l1_penalty", wl.radius)
    AtA, Atb = wl.A.T @ wl.A, wl.A.T @ wl.b
    grad = Atb - AtA @ xo
    S = xo != 0
    assert 0 < S.sum() < wl.d        # the weight zeroes some coefficients
    assert np.allclose(grad[S], wl.radius * np.sign(xo[S]), rtol=1e-9)
    assert np.all(np.abs(grad[~S]) <= wl.radius * (1 + 1e-9))
    xs = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=14, constraint="l1_penalty",
               radius=wl.radius)
    errs = [O.error_A(wl.A, x, xo) for x in xs[1:]]
    assert errs[-1] < 1e-8
    assert errs[6] < errs[0] * 1e-2


# ---------------------------------- one fixed sketch + conjugate gradients ----
def test_fixed_sketch_cg_collision_free_is_one_step():
    """With no bucket collisions H = A^T A, so the preconditioned residual is
    the Newton step and the first iterate is x_OPT."""
    g = np.random.default_rng(41)
    n, d, m = 12, 4, 1 << 22
    A = g.standard_normal((n, d))
    b = g.standard_normal(n)
    bucket, _ = sketch_hash(3, 0, n, m, 1)
    assert len(np.unique(bucket)) == n
    xs = O.fixed_sketch_cg(A, b, m, seed=3, iters=2)
    xo = O.x_opt(A, b)
    assert np.allclose(xs[1], xo, rtol=1e-12, atol=1e-13)


def test_fixed_sketch_cg_finite_termination_and_monotone_error():
    """Conjugate gradients end in at most d iterations in exact arithmetic,
    and the A^T A-norm of the error never grows (CG minimises it over the
    Krylov space); the Chebyshev bound 2 ((sqrt k - 1)/(sqrt k + 1))^t holds
    with k the condition number of H^{-1} A^T A."""
    g = np.random.default_rng(42)
    n, d, m = 400, 6, 24
    A = g.standard_normal((n, d)) * np.linspace(1, 30, d)
    b = g.standard_normal(n)
    xs = O.fixed_sketch_cg(A, b, m, seed=5, iters=d)
    xo = O.x_opt(A, b)
    err = [O.error_A(A, x, xo) for x in xs]
    assert err[d] < 1e-10 * err[0]
    assert all(err[t + 1] <= err[t] * (1 + 1e-9) for t in range(d))
    from oracle.sketch import sketch_apply_dense
    SA = sketch_apply_dense(A, 5, 0, m, 1)
    ev = sla_eigh(A.T @ A, SA.T @ SA)
    kappa = ev.max() / ev.min()
    rate = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    for t in range(1, d):
        assert err[t] <= 2 * rate ** t * err[0] * (1 + 1e-9), t


def sla_eigh(a, b):
    import scipy.linalg as sla
    return sla.eigh(a, b, eigvals_only=True)


def test_fixed_sketch_cg_fewer_passes_than_ihs():
    """On a tall problem with m = 8 d the preconditioned system is well
    conditioned, and CG contracts faster per pass over A than IHS with fresh
    sketches (0.32 against 0.43 per step here; the point of the variant);
    CSR input gives the same iterates as its dense copy."""
    wl = W.ols_dense(rows=20000, d=50, m=400, iters=12)
    xo = O.x_opt(wl.A, wl.b)
    cg = O.fixed_sketch_cg(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=12)
    ih = O.ihs(wl.A, wl.b, wl.m, seed=wl.sketch_seed, iters=12)
    e_cg = O.error_A(wl.A, cg[12], xo)
    e_ih = O.error_A(wl.A, ih[12], xo)
    assert e_cg < 1e-5 and e_cg < 0.1 * e_ih
    import scipy.sparse as sp
    C = sp.csr_matrix(wl.A[:3000])
    csr = (C.indptr.astype(np.int32), C.indices.astype(np.int32), C.data, 3000, wl.d)
    xd = O.fixed_sketch_cg(wl.A[:3000], wl.b[:3000], 100, seed=4, iters=5)
    xc = O.fixed_sketch_cg(None, wl.b[:3000], 100, seed=4, iters=5, csr=csr)
    for t in range(6):
        assert np.allclose(xd[t], xc[t], rtol=1e-12, atol=1e-14)
