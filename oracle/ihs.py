"""Oracle: the quantities one Iterative Hessian Sketch step needs, the QP of
Eq.(2) over the three constraint sets, the outer loop, the optimum x_OPT of
Eq.(1), the error metric of Def. A.1, and the derivative of the solution.

Everything is float64 numpy/scipy, written for a reader to check against the
paper by eye. No blocking, fusion or reordering beyond the definitions.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .dense_sketch import sketch_apply_gaussian, sketch_apply_srht
from .sketch import sketch_apply_csr, sketch_apply_dense, round_output


# --------------------------------------------------------------------------
# QP data (Sec. 1, the discussion after Eq.(2); App. A.1.1 "Iteration Time
# Costs"): the approximate Hessian (SA)^T SA and the inner-product terms
# --------------------------------------------------------------------------
def gram(SA):
    """H = (SA)^T (SA), the sketched Hessian."""
    SA = np.asarray(SA, dtype=np.float64)
    return SA.T @ SA


def gram_mixed(SA64, in_dtype):
    """Gram of SA rounded once to `in_dtype` (float32 / bfloat16), then formed
    in float64. The float64 product of two rounded inputs is the reference a
    reduced-precision Gram is compared with."""
    return gram(round_output(SA64, in_dtype).astype(np.float64))


def gradient(A, b, x):
    """Residual r = b - A x, gradient-side term g = A^T r (the linear term of
    Eq.(2)), and objective f = 1/2 ||r||^2 of Eq.(1)."""
    r = np.asarray(b, dtype=np.float64) - A @ x
    g = A.T @ r
    f = 0.5 * float(r @ r)
    return r, np.asarray(g, dtype=np.float64), f


def csr_matrix(indptr, indices, data, n, d):
    return sp.csr_matrix((np.asarray(data, dtype=np.float64),
                          np.asarray(indices), np.asarray(indptr)), shape=(n, d))


# --------------------------------------------------------------------------
# QP solvers: minimise 1/2 x^T H x - c^T x over C  (Eq.(2) with
# c = H x^t + g; the ball constraints are those of Eq.(1))
# --------------------------------------------------------------------------
class NotPositiveDefinite(ValueError):
    pass


def cholesky_solve(H, v):
    try:
        cf = sla.cho_factor(H, lower=True)
    except np.linalg.LinAlgError as e:
        raise NotPositiveDefinite(str(e))
    return sla.cho_solve(cf, v)


def project_l1_ball(v, tau):
    """Euclidean projection onto {x : ||x||_1 <= tau}: the sort-based method of
    Duchi, Shalev-Shwartz, Singer and Chandra (ICML 2008)."""
    v = np.asarray(v, dtype=np.float64)
    if np.abs(v).sum() <= tau:
        return v.copy()
    u = np.sort(np.abs(v))[::-1]
    css = np.cumsum(u)
    j = np.arange(1, len(u) + 1)
    rho = np.nonzero(u - (css - tau) / j > 0)[0][-1]
    theta = (css[rho] - tau) / (rho + 1.0)
    return np.sign(v) * np.maximum(np.abs(v) - theta, 0.0)


def l1_kkt_polish(H, c, tau, x):
    """Given a candidate x on the ball surface, solve the KKT system restricted
    to its support S and signs sigma:
        H_SS x_S + mu sigma = c_S,   sigma^T x_S = tau,
    and accept the result when it keeps the signs, has mu >= 0 and satisfies
    |c_j - (H x)_j| <= mu off the support. Returns (x, mu) or None."""
    S = np.nonzero(x)[0]
    if len(S) == 0:
        return None
    sig = np.sign(x[S])
    try:
        cf = sla.cho_factor(H[np.ix_(S, S)], lower=True)
    except np.linalg.LinAlgError:
        return None
    u = sla.cho_solve(cf, c[S])
    w = sla.cho_solve(cf, sig)
    mu = (sig @ u - tau) / (sig @ w)
    xs = u - mu * w
    if mu < 0 or np.any(np.sign(xs) != sig):
        return None
    out = np.zeros_like(x)
    out[S] = xs
    grad = c - H @ out
    off = np.ones(len(x), dtype=bool)
    off[S] = False
    scale = max(1.0, float(np.abs(c).max()))
    if off.any() and np.abs(grad[off]).max() > mu + 1e-9 * scale:
        return None
    return out, float(mu)


def qp_l1(H, c, tau, x0=None, max_iter=20000, tol=1e-15):
    """min 1/2 x^T H x - c^T x  s.t. ||x||_1 <= tau  (H positive definite).

    Inactive ball: the unconstrained minimiser. Otherwise accelerated projected
    gradient (FISTA with step 1/lambda_max(H) and function-value restart)
    identifies the support and signs, and the KKT polish solves the face
    exactly."""
    H = np.asarray(H, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    x_unc = cholesky_solve(H, c)
    if np.abs(x_unc).sum() <= tau:
        return x_unc
    L = float(np.linalg.eigvalsh(H)[-1])
    x = project_l1_ball(np.zeros_like(c) if x0 is None else x0, tau)
    y, tk = x.copy(), 1.0
    obj = lambda z: 0.5 * z @ (H @ z) - c @ z
    f_prev = obj(x)
    for _ in range(max_iter):
        x_new = project_l1_ball(y - (H @ y - c) / L, tau)
        f_new = obj(x_new)
        if f_new > f_prev:                   # restart the momentum
            y, tk = x.copy(), 1.0
            continue
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tk * tk))
        y = x_new + ((tk - 1.0) / t_new) * (x_new - x)
        step = np.abs(x_new - x).max()
        x, tk, f_prev = x_new, t_new, f_new
        if step <= tol * max(1.0, np.abs(x).max()):
            break
    pol = l1_kkt_polish(H, c, tau, x)
    return pol[0] if pol is not None else x


def soft_threshold(v, t):
    """The proximal map of t ||.||_1: sign(v_j) max(|v_j| - t, 0) componentwise."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def l1_penalty_kkt_polish(H, c, lam, x):
    """Given a candidate x, solve the optimality conditions of
    1/2 x^T H x - c^T x + lam ||x||_1 restricted to its support S and signs
    sigma:  H_SS x_S = c_S - lam sigma,  and accept the result when it keeps
    the signs and |c_j - (H x)_j| <= lam off the support. An empty support is
    accepted when |c_j| <= lam for every j. Returns x or None."""
    S = np.nonzero(x)[0]
    scale = max(1.0, float(np.abs(c).max()))
    if len(S) == 0:
        return np.zeros_like(x) if np.abs(c).max() <= lam + 1e-9 * scale else None
    sig = np.sign(x[S])
    try:
        cf = sla.cho_factor(H[np.ix_(S, S)], lower=True)
    except np.linalg.LinAlgError:
        return None
    xs = sla.cho_solve(cf, c[S] - lam * sig)
    if np.any(np.sign(xs) != sig):
        return None
    out = np.zeros_like(x)
    out[S] = xs
    grad = c - H @ out
    off = np.ones(len(x), dtype=bool)
    off[S] = False
    if off.any() and np.abs(grad[off]).max() > lam + 1e-9 * scale:
        return None
    return out


def qp_l1_penalty(H, c, lam, x0=None, max_iter=20000, tol=1e-15):
    """min 1/2 x^T H x - c^T x + lam ||x||_1  (H positive definite): the
    penalised form of the LASSO step that the experiments of Sec. 3 solve
    (lambda = 5). Accelerated proximal gradient (FISTA with step
    1/lambda_max(H), the soft threshold as the proximal map, function-value
    restart) identifies the support and signs, and the KKT polish solves the
    restricted optimality conditions exactly."""
    H = np.asarray(H, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    if np.abs(c).max() <= lam:           # 0 satisfies the optimality conditions
        return np.zeros_like(c)
    L = float(np.linalg.eigvalsh(H)[-1])
    x = np.zeros_like(c) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    y, tk = x.copy(), 1.0
    obj = lambda z: 0.5 * z @ (H @ z) - c @ z + lam * np.abs(z).sum()
    f_prev = obj(x)
    for _ in range(max_iter):
        x_new = soft_threshold(y - (H @ y - c) / L, lam / L)
        f_new = obj(x_new)
        if f_new > f_prev:                   # restart the momentum
            y, tk = x.copy(), 1.0
            continue
        t_new = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * tk * tk))
        y = x_new + ((tk - 1.0) / t_new) * (x_new - x)
        step = np.abs(x_new - x).max()
        x, tk, f_prev = x_new, t_new, f_new
        if step <= tol * max(1.0, np.abs(x).max()):
            break
    pol = l1_penalty_kkt_polish(H, c, lam, x)
    return pol if pol is not None else x


def qp_l2(H, c, radius):
    """min 1/2 x^T H x - c^T x  s.t. ||x||_2 <= radius  (H positive definite).

    If the unconstrained minimiser lies in the ball it is the answer; otherwise
    x(mu) = (H + mu I)^{-1} c with the unique mu > 0 at which ||x(mu)|| equals
    the radius, found by bisection on the eigen-decomposed secular function
    ||diag(1/(lambda + mu)) Q^T c||, which decreases monotonically in mu."""
    H = np.asarray(H, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    x_unc = cholesky_solve(H, c)
    if np.linalg.norm(x_unc) <= radius:
        return x_unc
    lam, Q = np.linalg.eigh(H)
    ch = Q.T @ c
    phi = lambda mu: np.linalg.norm(ch / (lam + mu))
    lo, hi = 0.0, np.linalg.norm(c) / radius
    while phi(hi) > radius:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if phi(mid) > radius:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    return cholesky_solve(H + mu * np.eye(len(c)), c)


def qp_step(H, g, x_t, constraint="none", radius=0.0):
    """One step of Eq.(2): argmin over C of
    1/2 (x - x^t)^T H (x - x^t) - g^T (x - x^t) = 1/2 x^T H x - (H x^t + g)^T x + const.
    For the penalised LASSO of Sec. 3 ("l1_penalty", radius = lambda) the
    regulariser lambda ||x||_1 is added to the sketched quadratic over all of
    R^d, the form of the step for a regularised objective."""
    if constraint == "none":
        return x_t + cholesky_solve(H, g)
    c = H @ x_t + g
    if constraint == "l1":
        return qp_l1(H, c, radius, x0=x_t)
    if constraint == "l2":
        return qp_l2(H, c, radius)
    if constraint == "l1_penalty":           # radius carries lambda
        return qp_l1_penalty(H, c, radius, x0=x_t)
    raise ValueError(constraint)


# --------------------------------------------------------------------------
# the outer loop (Eq.(2); Thm 2.2) and the optimum (Eq.(1))
# --------------------------------------------------------------------------
def ihs(A, b, m, s=1, seed=0, iter0=0, iters=10, constraint="none", radius=0.0,
        x0=None, csr=None, sketch_dtype="float64", return_hessians=False, kind="sparse"):
    """Run `iters` IHS steps from x0 (default 0). Step t draws the sketch keyed
    (seed, iter0 + t); x^{t+1} solves Eq.(2) with that sketch.
    Dense input: A (n x d). CSR input: A is ignored and csr = (indptr, indices,
    data, n, d). kind: "sparse" (CountSketch, or SJLT with s blocks), or one of
    the dense sketches "srht" and "gaussian" (Sec. 2) applied to A's rows.
    Returns the iterates x^0 .. x^iters (and the Hessians)."""
    if csr is not None:
        indptr, indices, data, n, d = csr
        Aop = csr_matrix(indptr, indices, data, n, d)
    else:
        Aop = np.asarray(A)
        n, d = Aop.shape
    A64 = Aop if csr is not None else Aop.astype(np.float64, copy=False)
    x = np.zeros(d) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    xs, Hs = [x.copy()], []
    dense_rows = None
    if kind != "sparse":
        dense_rows = A64.toarray() if csr is not None else A64
    for t in range(iters):
        if kind == "srht":
            SA = sketch_apply_srht(dense_rows, seed, iter0 + t, m, out_dtype=sketch_dtype)
        elif kind == "gaussian":
            SA = sketch_apply_gaussian(dense_rows, seed, iter0 + t, m, out_dtype=sketch_dtype)
        elif csr is not None:
            SA = sketch_apply_csr(indptr, indices, data, n, d, seed, iter0 + t,
                                  m, s, out_dtype=sketch_dtype)
        else:
            SA = sketch_apply_dense(Aop, seed, iter0 + t, m, s,
                                    out_dtype=sketch_dtype)
        H = gram(np.asarray(SA, dtype=np.float64))
        _, g, _ = gradient(A64, b, x)
        x = qp_step(H, g, x, constraint, radius)
        xs.append(x.copy())
        Hs.append(H)
    return (xs, Hs) if return_hessians else xs


def fixed_sketch_cg(A, b, m, s=1, seed=0, iter0=0, iters=10, x0=None, csr=None,
                    problem=0):
    """The reduced-data-access variant the paper's conclusion points to, for
    C = R^d: one sketch S (key (seed, iter0)) is drawn once, and its Hessian
    sketch H = (SA)^T SA preconditions conjugate gradients on the normal
    equations A^T A x = A^T b (preconditioned CG as in Hestenes and Stiefel,
    1952; the preconditioner enters through z = H^{-1} r). Each iteration
    reads A twice here (A p, then A^T (A p)); the GPU forms A^T A p in one
    pass. Returns the iterates x^0 .. x^iters.

    The steps, from x^0 (default 0):
        r = A^T (b - A x^0),  z = H^{-1} r,  p = z,  rho = r^T z
        repeat: q = A^T A p,  alpha = rho / p^T q,  x += alpha p,
                r -= alpha q,  z = H^{-1} r,  rho' = r^T z,
                p = z + (rho' / rho) p,  rho = rho'
    """
    if csr is not None:
        indptr, indices, data, n, d = csr
        Aop = csr_matrix(indptr, indices, data, n, d)
        SA = sketch_apply_csr(indptr, indices, data, n, d, seed, iter0, m, s, problem=problem)
    else:
        Aop = np.asarray(A, dtype=np.float64)
        n, d = Aop.shape
        SA = sketch_apply_dense(Aop, seed, iter0, m, s, problem=problem)
    H = gram(SA)
    factor = sla.cho_factor(H, lower=True)
    x = np.zeros(d) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r = Aop.T @ (np.asarray(b, dtype=np.float64) - Aop @ x)
    z = sla.cho_solve(factor, r)
    p = z.copy()
    rho = float(r @ z)
    xs = [x.copy()]
    for _ in range(iters):
        q = Aop.T @ (Aop @ p)
        pq = float(p @ q)
        alpha = rho / pq if rho != 0.0 else 0.0
        x = x + alpha * p
        r = r - alpha * q
        z = sla.cho_solve(factor, r)
        rho_new = float(r @ z)
        beta = rho_new / rho if rho != 0.0 else 0.0
        p = z + beta * p
        rho = rho_new
        xs.append(x.copy())
    return xs


def x_opt(A, b, constraint="none", radius=0.0):
    """x_OPT of Eq.(1), or of the penalised LASSO of Sec. 3 ("l1_penalty",
    radius = lambda). A dense array or a scipy sparse matrix."""
    if constraint == "none":
        if sp.issparse(A):
            A = A.toarray()
        return np.linalg.lstsq(np.asarray(A, dtype=np.float64), b, rcond=None)[0]
    AtA = A.T @ A
    AtA = AtA.toarray() if sp.issparse(AtA) else AtA
    Atb = np.asarray(A.T @ b).ravel()
    if constraint == "l1":
        return qp_l1(AtA, Atb, radius)
    if constraint == "l2":
        return qp_l2(AtA, Atb, radius)
    if constraint == "l1_penalty":           # 1/2 ||Ax - b||^2 + lambda ||x||_1
        return qp_l1_penalty(AtA, Atb, radius)
    raise ValueError(constraint)


def error_A(A, x, x_ref):
    """Relative error in the prediction seminorm of Sec. 1 / Def. A.1:
    ||x - x_OPT||_A / ||x_OPT||_A = ||A (x - x_OPT)|| / ||A x_OPT|| (the 1/sqrt(n)
    factors cancel)."""
    return float(np.linalg.norm(A @ (x - x_ref)) / np.linalg.norm(A @ x_ref))


def error_euclid(x, x_ref):
    return float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref))


# --------------------------------------------------------------------------
# derivative of the unconstrained solution (implicit differentiation of the
# normal equations A^T A x = A^T b); loss L = ||x - y||^2
# --------------------------------------------------------------------------
def loss_and_grads_closed_form(A, b, y):
    """L(x_OPT(A, b)) and its exact gradients with respect to b and A:
         xbar = 2 (x - y),  lambda = (A^T A)^{-1} xbar,
         dL/db = A lambda,   dL/dA = r lambda^T - (A lambda) x^T,  r = b - A x.
    lambda is formed from the R factor of a QR of A (no squared condition)."""
    A = np.asarray(A, dtype=np.float64)
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    R = np.linalg.qr(A, mode="r")
    xbar = 2.0 * (x - y)
    lam = sla.solve_triangular(R, sla.solve_triangular(R.T, xbar, lower=True))
    r = b - A @ x
    Al = A @ lam
    return float(np.sum((x - y) ** 2)), Al, np.outer(r, lam) - np.outer(Al, x)


def adjoint_ihs(A, Hs, xbar):
    """lambda from A^T A lambda = xbar by the IHS-preconditioned iteration
    lambda <- lambda + H_k^{-1} (xbar - A^T A lambda), one step per forward
    Hessian H_k, in the forward's order, from lambda = 0."""
    A = np.asarray(A, dtype=np.float64)
    lam = np.zeros(A.shape[1])
    for H in Hs:
        resid = xbar - A.T @ (A @ lam)
        lam = lam + cholesky_solve(H, resid)
    return lam


def grads_from_lambda(A, b, x, lam):
    """dL/db = A lambda and dL/dA = r lambda^T - (A lambda) x^T, r = b - A x."""
    A = np.asarray(A, dtype=np.float64)
    r = b - A @ x
    Al = A @ lam
    return Al, np.outer(r, lam) - np.outer(Al, x)
