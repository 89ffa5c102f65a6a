"""The allocation-free sketch apply (ihs_sketch_apply_static, for callers
that cannot allocate device memory) against the workspace entry point
ihs_sketch_apply: the same S A bit for bit (the sketch is integer-exact
work: the sequential-order bucket sums), on two calls in a row whose second
input is smaller, so the shared scratch array's leftovers from the first
call must not leak into the second."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_static_scratch_matches_workspace_entry_point(gpu_lib):
    import torch
    P = gpu_lib
    g = np.random.default_rng(77)
    big = g.standard_normal((1 << 18, 96))
    small = g.standard_normal((3001, 40))
    wl = W.ridge_csr(rows=20000, d=200, density=0.01)
    csr = P.Matrix(row_ptr=dev(wl.indptr), col_idx=dev(wl.indices), values=dev(wl.data),
                   n=wl.n, d=wl.d)
    cases = [
        (P.Matrix(dense=dev(big)), P.SketchSpec(4096, seed=5, iter=2), "float64"),
        (P.Matrix(dense=dev(small)), P.SketchSpec(400, s=4, kind="sjlt", seed=9), "float32"),
        (csr, P.SketchSpec(1000, seed=3, iter=1), "float64"),
        (P.Matrix(dense=dev(small[:17])), P.SketchSpec(64, seed=1), "bfloat16"),
    ]
    for A, sk, dt in cases:
        # poisoned outputs: every entry must be written
        out = torch.full((A.batch * sk.m, A.d), float("nan"), dtype=getattr(torch, dt),
                         device="cuda")
        P.sketch_apply_static(A, sk, dt, out=out)
        ref = P.sketch_apply(A, sk, dt)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int16 if dt == "bfloat16" else
                                    (torch.int32 if dt == "float32" else torch.int64)),
                           ref.view(torch.int16 if dt == "bfloat16" else
                                    (torch.int32 if dt == "float32" else torch.int64))), (sk, dt)


def test_static_scratch_headline_size_fits(gpu_lib):
    """The headline sketch (CountSketch, m = 4096) over 2^22 rows fits the
    scratch array; checked here on a 2^22 x 8 matrix against the workspace
    entry point."""
    import torch
    P = gpu_lib
    A = torch.randn(1 << 22, 8, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(4))
    M = P.Matrix(dense=A)
    sk = P.SketchSpec(4096, seed=11, iter=3)
    out = P.sketch_apply_static(M, sk)
    ref = P.sketch_apply(M, sk)
    assert torch.equal(out.view(torch.int64), ref.view(torch.int64))
