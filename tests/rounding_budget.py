"""Rounding budgets: how far two correct float64 implementations of the same
IHS run (Eq.(2), the same sketches) may drift apart.

Both implementations compute the same exact quantities; they differ only in
the order of their floating-point sums and in how they solve the d x d
system. The budget follows each rounding source to the iterate and carries it
through the later steps, so a tolerance is a consequence of the arithmetic
and of the problem's conditioning, not a guess.

The rounding model (Higham and Mary, "A new approach to probabilistic
rounding error analysis", SIAM J. Sci. Comput. 41, 2019): every rounding is
an independent error of relative size at most u = 2^-53 with mean zero, so
the error of a sum of k terms, taken in any order, has variance at most
u^2 times the sum over its k roundings of the squared partial sum each
rounds. Per step t, with x = x^t, delta = x^{t+1} - x^t, M = A^T A:

  Gram     H_ij = sum of m products; partial sums are at most
           S_ij = sum_k |SA_ki| |SA_kj|, so var(dH_ij) <= m u_g^2 S_ij^2, with
           u_g the unit roundoff of the Gram's accumulation (u, or 2^-24 for
           a float32 accumulation of inputs rounded identically on both
           sides, whose products are exact). The step's response to dH is
           dx = -P dH delta (P below).
  gradient g_i = sum over the n rows of A_ri r_r. The rows are i.i.d. draws
           and every summation order here is independent of their values,
           so the terms are exchangeable and a partial sum over k of them has
           second moment k^2 mu^2 + k v (mean mu = g_i / n, variance v); over
           any summation tree, var(dg_i) <= u^2 n (g_i^2 + sum_r (A_ri r_r)^2).
  residual r_r = b_r - A_r x carries an error of variance at most
           d u^2 (|b_r| + |A_r||x|)^2, which reaches g as A^T (those errors):
           covariance A^T diag(.) A.
  solve    a backward-stable Cholesky solve of the d x d (or face) system
           meets (K + dK) z = rhs with |dK| <= gamma_{3k+1} |L||L^T|
           (Higham, Thm 10.4); the probabilistic form replaces gamma_{3k+1}
           by sqrt(3k+1) u. The unconstrained step responds with
           -H^{-1} dH delta; a constrained step that solves for x^{t+1} on
           its face with -P dK x^{t+1}.
  c        the constrained steps form c = H x + g first: variance at most
           d u^2 (sum_j |H_ij x_j| + |g_i|)^2 per entry.

P is the derivative of the step's solution with respect to c: H^{-1} for
C = R^d and inactive balls; on the face F (support and signs sigma) of an
l1-ball solution, H_FF^{-1} - H_FF^{-1} sigma sigma^T H_FF^{-1} / (sigma^T
H_FF^{-1} sigma); H_FF^{-1} on the face of a penalised solution; for an
active l2 ball, R - R x x^T R / (x^T R x) with R = (H + mu I)^{-1}.

The difference D_t of the two runs' iterates then obeys, to first order,
D_{t+1} = T_t D_t + xi_t with T_t = P (H_t - M) (= I - H_t^{-1} M for
C = R^d: the exact IHS error recurrence) and xi_t carrying both runs'
rounding, so its covariance C_t propagates exactly:
C_{t+1} = T_t C_t T_t^T + 2 P Xi_t P^T, Xi_t the per-run covariance above.
The budget of iterate t is LAMBDA standard deviations: LAMBDA sqrt(tr(M C_t))
in the prediction norm ||A .|| of Def. A.1 and LAMBDA sqrt(tr(C_t)) in the
Euclidean norm. Chebyshev's inequality puts the chance of exceeding it at
most 1/LAMBDA^2 under the model; the model itself overstates the partial
sums of the Gram (S_ij) and of the solve.

This is test infrastructure. It reads the oracle's iterates and Hessians and
never the library's.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

U = 2.0 ** -53
LAMBDA = 10.0


def _dense(X):
    return X.toarray() if sp.issparse(X) else np.asarray(X)


def face_projector(H, c, x_next, constraint, radius):
    """P of the step whose solution (from the oracle) is x_next. Returns the
    d x d matrix P and the matrix K whose backward error the final solve of
    that step carries (None for the unconstrained step, whose solve responds
    to delta instead)."""
    d = len(c)
    if constraint == "none":
        return sla.cho_solve(sla.cho_factor(H, lower=True), np.eye(d)), None
    if constraint == "l2":
        nx = np.linalg.norm(x_next)
        if nx < radius * (1 - 1e-9):        # inactive: the unconstrained minimiser
            return sla.cho_solve(sla.cho_factor(H, lower=True), np.eye(d)), H
        mu = float((c - H @ x_next) @ x_next) / (nx * nx)
        K = H + max(mu, 0.0) * np.eye(d)
        R = sla.cho_solve(sla.cho_factor(K, lower=True), np.eye(d))
        Rx = R @ x_next
        return R - np.outer(Rx, Rx) / float(x_next @ Rx), K
    F = np.nonzero(x_next)[0]
    P = np.zeros((d, d))
    if len(F) == 0:
        return P, None
    HF = H[np.ix_(F, F)]
    RF = sla.cho_solve(sla.cho_factor(HF, lower=True), np.eye(len(F)))
    if constraint == "l1" and np.abs(x_next).sum() >= radius * (1 - 1e-12):
        sg = np.sign(x_next[F])
        Rs = RF @ sg
        RF = RF - np.outer(Rs, Rs) / float(sg @ Rs)
    elif constraint == "l1" and np.abs(x_next).sum() < radius * (1 - 1e-12):
        # inactive ball: the unconstrained minimiser on all of R^d
        return sla.cho_solve(sla.cho_factor(H, lower=True), np.eye(d)), H
    P[np.ix_(F, F)] = RF
    K = np.zeros((d, d))
    K[np.ix_(F, F)] = HF
    return P, K


def _solve_var(K, z):
    """Per-entry variance of dK z for a backward-stable Cholesky solve of K
    (zero rows and columns of K, outside a face, carry no error)."""
    live = np.nonzero(np.abs(np.diag(K)) > 0)[0]
    v = np.zeros(len(z))
    if len(live) == 0:
        return v
    Kl = K[np.ix_(live, live)]
    L = np.linalg.cholesky(Kl)
    LL = np.abs(L) @ np.abs(L).T
    k = len(live)
    v[live] = (3 * k + 1) * U * U * ((LL ** 2) @ (z[live] ** 2))
    return v


def step_covariance(A, b, SA, H, x, x_next, constraint, radius, sa_err=None, gram_u=U):
    """(P, T, Xi): the step's derivative with respect to c, the error map T
    and one run's rounding covariance Xi (before P) of one IHS step.
    sa_err (optional, m x d): a bound on |dSA| when the two runs' sketches
    are not bitwise equal (the Gaussian sketch, whose entries come from
    transcendental functions); it enters H as |dSA|^T |SA| + |SA|^T |dSA|,
    counted in full as a standard deviation. gram_u: the unit roundoff of the
    Gram's accumulation in the run compared (u_g above)."""
    n, d = A.shape
    m = SA.shape[0]
    M = _dense(A.T @ A)
    r = b - A @ x
    g = np.asarray(A.T @ r).ravel()
    c = H @ x + g
    P, K = face_projector(H, c, x_next, constraint, radius)
    T = P @ (H - M)
    delta = x_next - x
    S = np.abs(SA).T @ np.abs(SA)
    v = m * gram_u * gram_u * ((S ** 2) @ (delta ** 2))            # Gram
    if sa_err is not None:
        E = sa_err.T @ np.abs(SA)
        v = v + ((E + E.T) ** 2) @ (delta ** 2)
    if sp.issparse(A):
        absA = abs(A)
        t2 = np.asarray(A.multiply(A).T @ (r * r)).ravel()
        rb = np.abs(b) + np.asarray(absA @ np.abs(x)).ravel()
        w = np.sqrt(d * U * U) * rb
        Aw = A.multiply(w[:, None]).tocsr()
        cov_res = _dense(Aw.T @ Aw)
    else:
        absA = np.abs(A)
        t2 = (A * A).T @ (r * r)
        rb = np.abs(b) + absA @ np.abs(x)
        Aw = A * (np.sqrt(d) * U * rb)[:, None]
        cov_res = Aw.T @ Aw
    v = v + n * U * U * (g * g + t2)                                # gradient sums
    if K is None:                                                    # unconstrained solve
        if constraint == "none":
            L = np.linalg.cholesky(H)
            LL = np.abs(L) @ np.abs(L).T
            v = v + (3 * d + 1) * U * U * ((LL ** 2) @ (delta ** 2))
    else:
        v = v + _solve_var(K, x_next)                                # face solve
        v = v + d * U * U * ((np.abs(H) @ np.abs(x) + np.abs(g)) ** 2)  # c = H x + g
    Xi = np.diag(v) + cov_res
    return P, T, Xi


def ihs_budget(A, b, sketches, hessians, iterates, constraint="none", radius=0.0,
               lam=LAMBDA, sketch_errs=None, gram_u=U):
    """Budgets for the iterates x^1 .. x^N of one IHS run: a list of
    (bound in ||A .||, bound in ||.||_2). sketches[t] and hessians[t] are the
    oracle's S_t A and H_t, iterates the oracle's x^0 .. x^N; sketch_errs[t]
    (optional) bounds |dSA| of step t (see step_covariance); gram_u the unit
    roundoff of the compared run's Gram accumulation (one of the two runs:
    the oracle's Gram is float64)."""
    d = len(iterates[0])
    M = _dense(A.T @ A)
    C = np.zeros((d, d))
    out = []
    for t in range(len(hessians)):
        x, xn = iterates[t], iterates[t + 1]
        P, T, Xi = step_covariance(A, b, sketches[t], hessians[t], x, xn, constraint, radius,
                                   None if sketch_errs is None else sketch_errs[t], gram_u)
        if gram_u != U:  # the oracle's own float64 Gram rounds at u
            _, _, Xi64 = step_covariance(A, b, sketches[t], hessians[t], x, xn, constraint,
                                         radius, None, U)
            C = T @ C @ T.T + P @ (Xi + Xi64) @ P.T + np.diag(2.0 * U * U * xn * xn)
        else:
            C = T @ C @ T.T + 2.0 * (P @ Xi @ P.T) + np.diag(2.0 * U * U * xn * xn)
        C = 0.5 * (C + C.T)
        out.append((lam * np.sqrt(max(np.trace(M @ C), 0.0)),
                    lam * np.sqrt(max(np.trace(C), 0.0))))
    return out


def qp_budget(H, g, x, x_next, constraint="none", radius=0.0, cg_tol=0.0, lam=LAMBDA):
    """Euclidean budget of one QP step computed twice from the same exact
    (H, g, x^t): the two runs differ by their formation of c and their final
    solve. cg_tol > 0 adds, for one run, a solve of the face system by
    conjugate gradients to relative residual cg_tol (deterministic, added to
    the bound: ||P|| cg_tol ||rhs||)."""
    d = len(g)
    c = H @ x + g
    P, K = face_projector(H, c, x_next, constraint, radius)
    delta = x_next - x
    if constraint == "none":
        L = np.linalg.cholesky(H)
        LL = np.abs(L) @ np.abs(L).T
        v = (3 * d + 1) * U * U * ((LL ** 2) @ (delta ** 2))
    else:
        v = d * U * U * ((np.abs(H) @ np.abs(x) + np.abs(g)) ** 2)
        if K is not None:
            v = v + _solve_var(K, x_next)
    Cov = 2.0 * (P @ np.diag(v) @ P.T) + np.diag(2.0 * U * U * x_next * x_next)
    bound = lam * np.sqrt(max(np.trace(Cov), 0.0))
    if cg_tol > 0 and constraint != "none":
        bound += np.linalg.norm(P, 2) * cg_tol * (np.linalg.norm(c) + np.linalg.norm(H @ x_next))
    return bound


def h_norm_budget(H, g, lam=LAMBDA):
    """Budget in the H-norm sqrt(v^T H v) for the unconstrained step
    delta = H^{-1} g computed twice by backward-stable solves: the response
    -H^{-1} dH delta has H-norm covariance sum_i (H^{-1})_ii var((dH delta)_i)."""
    d = len(g)
    cf = sla.cho_factor(H, lower=True)
    delta = sla.cho_solve(cf, g)
    L = np.tril(cf[0])
    LL = np.abs(L) @ np.abs(L).T
    v = (3 * d + 1) * U * U * ((LL ** 2) @ (delta ** 2))
    Hi_diag = np.diag(sla.cho_solve(cf, np.eye(d)))
    return lam * np.sqrt(2.0 * float(Hi_diag @ v))
