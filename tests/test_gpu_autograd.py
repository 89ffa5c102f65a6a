"""The differentiation extension: torch.autograd functions over the library.

SketchApply's backward is the adjoint S^T G (bit-exact against the oracle's
adjoint, and gradcheck-pinned since S is linear). IHSSolve's backward is the
implicit derivative of x_OPT for the unconstrained problem: it is checked
against the float64 closed form (QR, no squared condition number), against
central finite differences of L(x_IHS(A, b)) with the sketch seeds fixed (the
hash ignores the values, so x_IHS is smooth in A and b), and by gradcheck on a
tiny problem where x_IHS equals x_OPT to rounding."""
import numpy as np
import pytest

import workloads as W
from oracle import ihs as O
from oracle import sketch as OS

pytestmark = pytest.mark.gpu


def dev(x, grad=False):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t.requires_grad_(grad)


def host(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("kind,s", [("countsketch", 1), ("sjlt", 2)])
def test_sketch_apply_backward_is_the_adjoint(gpu_lib, kind, s):
    import torch
    from paper_1910_14166_amd import autograd as AG
    g = np.random.default_rng(3)
    n, d, m = 3000, 24, 64
    A = g.standard_normal((n, d))
    W_ = g.standard_normal((m, d))
    At = dev(A, True)
    SA = AG.sketch(At, m, s=s, kind=kind, seed=5, iter=2)
    (SA * dev(W_)).sum().backward()
    want = OS.sketch_adjoint(W_, n, seed=5, iteration=2, m=m, s=s)
    assert np.array_equal(host(At.grad), want)
    assert np.array_equal(host(SA), OS.sketch_apply_dense(A, 5, 2, m, s))
    # gradcheck on a tiny instance (S is linear: finite differences are exact)
    At2 = dev(g.standard_normal((40, 3)), True)
    assert torch.autograd.gradcheck(lambda a: AG.sketch(a, 8, s=s, kind=kind, seed=1), (At2,),
                                    eps=1e-6, atol=1e-9)


def test_ihs_solve_grads_match_closed_form(gpu_lib):
    from paper_1910_14166_amd import autograd as AG
    g = np.random.default_rng(4)
    n, d = 4000, 16
    A = g.standard_normal((n, d))
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    y = g.standard_normal(d)
    At, bt = dev(A, True), dev(b, True)
    x = AG.ihs_solve(At, bt, m=160, seed=11, iters=40)
    ((x[0] - dev(y)) ** 2).sum().backward()
    _, db, dA = O.loss_and_grads_closed_form(A, b, y)
    assert np.linalg.norm(host(bt.grad) - db) <= 1e-9 * np.linalg.norm(db)
    assert np.linalg.norm(host(At.grad) - dA) <= 1e-9 * np.linalg.norm(dA)


def test_ihs_solve_grads_match_finite_differences(gpu_lib):
    import torch
    from paper_1910_14166_amd import autograd as AG
    g = np.random.default_rng(5)
    n, d, m, seed, iters = 2000, 10, 100, 21, 45
    A = g.standard_normal((n, d))
    b = A @ g.standard_normal(d) + 0.1 * g.standard_normal(n)
    y = g.standard_normal(d)

    def loss(Av, bv):
        x = AG.ihs_solve(Av, bv, m=m, seed=seed, iters=iters)
        return ((x[0] - dev(y)) ** 2).sum()

    At, bt = dev(A, True), dev(b, True)
    loss(At, bt).backward()
    gA, gb = host(At.grad), host(bt.grad)
    with torch.no_grad():
        for k in range(4):
            E = g.standard_normal((n, d))
            e = g.standard_normal(n)
            h = 1e-5
            fd_a = (float(loss(dev(A + h * E), dev(b))) - float(loss(dev(A - h * E), dev(b)))) / (2 * h)
            fd_b = (float(loss(dev(A), dev(b + h * e))) - float(loss(dev(A), dev(b - h * e)))) / (2 * h)
            assert abs(fd_a - np.sum(gA * E)) <= 1e-6 * max(1.0, abs(fd_a)), k
            assert abs(fd_b - gb @ e) <= 1e-6 * max(1.0, abs(fd_b)), k


def test_ihs_solve_gradcheck_tiny(gpu_lib):
    import torch
    from paper_1910_14166_amd import autograd as AG
    g = np.random.default_rng(6)
    A = dev(g.standard_normal((64, 3)), True)
    b = dev(g.standard_normal(64), True)
    assert torch.autograd.gradcheck(lambda a, bb: AG.ihs_solve(a, bb, m=24, seed=2, iters=80),
                                    (A, b), eps=1e-6, atol=1e-6, rtol=1e-4)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_ragged_batch_grads(gpu_lib, dtype):
    from paper_1910_14166_amd import autograd as AG
    wl = W.batch_ragged(num=6, n_lo=2000, n_hi=6000, d=64, iters=30, dtype=dtype)
    At, bt = dev(wl.A, True), dev(wl.b, True)
    x = AG.ihs_solve(At, bt, m=wl.m, seed=wl.sketch_seed, iters=wl.iters,
                     row_offsets=wl.row_offsets)
    ((x - dev(wl.y)) ** 2).sum().backward()
    gA, gb = host(At.grad), host(bt.grad)
    A64 = wl.A.astype(np.float64)
    tol = 1e-8 if dtype == "float64" else 1e-6
    for p in range(wl.batch):
        r0, r1 = wl.row_offsets[p], wl.row_offsets[p + 1]
        _, db, dA = O.loss_and_grads_closed_form(A64[r0:r1], wl.b[r0:r1], wl.y[p])
        assert np.linalg.norm(gb[r0:r1] - db) <= tol * np.linalg.norm(db), p
        assert np.linalg.norm(gA[r0:r1] - dA) <= tol * np.linalg.norm(dA), p


def test_ragged_batch_grads_full_size_sampled(gpu_lib):
    """The differentiation workload at full size (64 problems, n in
    [16384, 131072], d = 64, m = 640, 20 steps), generated on the device; the
    closed form is computed for three sampled problems."""
    import torch
    from paper_1910_14166_amd import autograd as AG
    wl = W.batch_ragged(backend="torch", device="cuda")
    At = wl.A.clone().requires_grad_(True)
    bt = wl.b.clone().requires_grad_(True)
    x = AG.ihs_solve(At, bt, m=wl.m, seed=wl.sketch_seed, iters=wl.iters,
                     row_offsets=wl.row_offsets)
    ((x - wl.y) ** 2).sum().backward()
    torch.cuda.synchronize()
    for p in (0, 31, 63):
        r0, r1 = int(wl.row_offsets[p]), int(wl.row_offsets[p + 1])
        A = wl.A[r0:r1].cpu().numpy()
        _, db, dA = O.loss_and_grads_closed_form(A, wl.b[r0:r1].cpu().numpy(),
                                                 wl.y[p].cpu().numpy())
        # 20 steps at m = 10 d contract the IHS error to about 1e-9
        assert np.linalg.norm(host(bt.grad[r0:r1]) - db) <= 1e-6 * np.linalg.norm(db), p
        assert np.linalg.norm(host(At.grad[r0:r1]) - dA) <= 1e-6 * np.linalg.norm(dA), p


def test_solution_grads_many_problems(gpu_lib):
    """ihs_solution_grads over more problems than one launch takes (70 > 64),
    with empty and one-row problems, for float64 and float32 data:
    dL/db = A lambda and dL/dA = r lambda^T - (A lambda) x^T per problem,
    against the same formulas in numpy (float64, within the rounding of
    d-term dot products)."""
    import torch
    P = gpu_lib
    g = np.random.default_rng(77)
    sizes = g.integers(0, 120, 70)
    sizes[[0, 33, 65]] = 0
    sizes[[2, 64]] = 1
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n, d = int(offs[-1]), 20
    for dt in (np.float64, np.float32):
        A = g.standard_normal((n, d)).astype(dt)
        b = g.standard_normal(n)
        x = g.standard_normal((70, d))
        lam = g.standard_normal((70, d))
        M = P.Matrix(dense=torch.from_numpy(A).cuda(), row_offsets=offs)
        db, dA = P.solution_grads(M, dev(b), dev(x), dev(lam))
        db, dA = host(db), host(dA)
        A64 = A.astype(np.float64)
        for p in range(70):
            r0, r1 = offs[p], offs[p + 1]
            Al = A64[r0:r1] @ lam[p]
            r = b[r0:r1] - A64[r0:r1] @ x[p]
            ref = np.outer(r, lam[p]) - np.outer(Al, x[p])
            scale = np.abs(A64[r0:r1]).sum(1, keepdims=True) + 1.0
            assert np.allclose(db[r0:r1], Al, rtol=0, atol=1e-13 * 20 * 10), p
            assert np.all(np.abs(dA[r0:r1] - ref) <= 1e-12 * scale * 10), p
