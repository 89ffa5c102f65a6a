"""torch.autograd wrappers over libihs (the differentiation extension).

SketchApply   SA = S A for a CountSketch/SJLT S (Sec. 2). S is a fixed linear
              map (the hash ignores the values), so the backward pass is the
              adjoint: dL/dA = S^T dL/d(SA), computed by ihs_sketch_adjoint
              with the same signs and 1/sqrt(s) scale.
IHSSolve      x = IHS(A, b) for the unconstrained problem of Eq.(1). The
              backward pass differentiates the solution x_OPT = (A^T A)^{-1} A^T b
              implicitly: lambda solves A^T A lambda = xbar (ihs_adjoint_solve,
              an IHS-preconditioned iteration reusing the forward's Cholesky
              factors), then dL/db = A lambda and
              dL/dA = r lambda^T - (A lambda) x^T with r = b - A x
              (ihs_solution_grads).

Both run entirely in the library's kernels; these classes only marshal
arguments. A ragged batch stacks the problems' rows (row_offsets, host list)
and returns x as (batch, d).
"""
from __future__ import annotations

import torch

from . import Matrix, SketchSpec, adjoint_solve, options, sketch_adjoint, sketch_apply, \
    solution_grads, solve


class SketchApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, spec: SketchSpec, row_offsets=None):
        if A.stride(1) != 1:
            A = A.contiguous()
        SA = sketch_apply(Matrix(dense=A, row_offsets=row_offsets), spec, out_dtype="float64")
        ctx.spec, ctx.row_offsets, ctx.n, ctx.a_dtype = spec, row_offsets, A.shape[0], A.dtype
        return SA

    @staticmethod
    def backward(ctx, g_sa):
        if not ctx.needs_input_grad[0]:
            return None, None, None
        g = sketch_adjoint(g_sa.contiguous().double(), ctx.n, ctx.spec,
                           row_offsets=ctx.row_offsets)
        return g.to(ctx.a_dtype), None, None


class IHSSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, b, m, seed=0, iters=20, s=1, kind="countsketch", row_offsets=None):
        if A.stride(1) != 1:
            A = A.contiguous()
        b = b.contiguous().double()
        M = Matrix(dense=A, row_offsets=row_offsets)
        opts = options(m, s=s, kind=kind, seed=seed, max_iter=iters)
        res = solve(M, b, opts, factors=True)
        ctx.save_for_backward(A, b, res.x, res.factors)
        ctx.row_offsets = row_offsets
        return res.x.clone()

    @staticmethod
    def backward(ctx, xbar):
        A, b, x, factors = ctx.saved_tensors
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_a or need_b):
            return (None,) * 8
        M = Matrix(dense=A, row_offsets=ctx.row_offsets)
        lam = adjoint_solve(M, xbar.contiguous().double(), factors)
        db, dA = solution_grads(M, b, x, lam, want_db=need_b, want_dA=need_a)
        if dA is not None:
            dA = dA.to(A.dtype)
        return dA, db, None, None, None, None, None, None


def sketch(A, m, s=1, kind="countsketch", seed=0, iter=0, row_offsets=None):
    """SA for a differentiable A (float64 output)."""
    return SketchApply.apply(A, SketchSpec(m, s, kind, seed, iter), row_offsets)


def ihs_solve(A, b, m, seed=0, iters=20, s=1, kind="countsketch", row_offsets=None):
    """x_IHS (batch x d) for differentiable A and b (unconstrained)."""
    return IHSSolve.apply(A, b, m, seed, iters, s, kind, row_offsets)
