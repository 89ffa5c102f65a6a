"""No entry point leaves a HIP error pending on the calling thread: after
each call (and a device synchronisation) the runtime's hipGetLastError
returns hipSuccess. The entry points clear errors that earlier, unrelated HIP
calls left pending before their own first launch, so a pending error after a
call could only be the library's own."""
import ctypes
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hip(gpu_lib):
    """The HIP runtime this process already uses (the one torch and the
    library share), found in the process's memory map: loading another copy
    from elsewhere would start a second runtime."""
    import torch
    torch.zeros(1, device="cuda")
    path = None
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64.so" in line:
                path = line.split()[-1]
                break
    assert path is not None, "no HIP runtime mapped"
    h = ctypes.CDLL(path, mode=os.RTLD_NOLOAD | ctypes.RTLD_GLOBAL)
    h.hipGetLastError.restype = ctypes.c_int
    h.hipDeviceSynchronize.restype = ctypes.c_int
    return h


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_entry_points_leave_no_pending_error(gpu_lib, hip):
    import torch
    P = gpu_lib
    wl = W.ols_dense(rows=5000, d=40, m=400, iters=4)
    A, b = dev(wl.A), dev(wl.b)
    M = P.Matrix(dense=A)
    csr = W.table1_like("w8a", rows=3000)
    Mc = P.Matrix(row_ptr=dev(csr.indptr), col_idx=dev(csr.indices), values=dev(csr.data),
                  n=csr.n, d=csr.d)
    x = torch.zeros(1, 40, dtype=torch.float64, device="cuda")
    ones = torch.ones(400, 40, dtype=torch.float64, device="cuda")
    eye = torch.eye(40, dtype=torch.float64, device="cuda")[None].contiguous()
    xp = x + 1.0
    calls = {
        "hash": lambda: P.sketch_hash(5000, P.SketchSpec(400)),
        "apply": lambda: P.sketch_apply(M, P.SketchSpec(400, seed=2)),
        "apply_csr": lambda: P.sketch_apply(Mc, P.SketchSpec(600, s=4, kind="sjlt")),
        "apply_static": lambda: P.sketch_apply_static(M, P.SketchSpec(400)),
        "apply_srht": lambda: P.sketch_apply(M, P.SketchSpec(400, kind="srht")),
        "apply_gaussian": lambda: P.sketch_apply(M, P.SketchSpec(100, kind="gaussian")),
        "adjoint": lambda: P.sketch_adjoint(ones, 5000, P.SketchSpec(400)),
        "gram": lambda: P.gram(ones, 400),
        "gradient": lambda: P.gradient(M, b, x),
        "qp_step": lambda: P.qp_step(eye, xp, x),
        "solve": lambda: P.solve(M, b, P.options(400, seed=1, max_iter=4)),
        "solve_tol": lambda: P.solve(M, b, P.options(400, seed=1, max_iter=30, tol=1e-6),
                                     raise_on_error=False),
        "read_ceiling": lambda: P.read_ceiling(A),
    }
    for name, fn in calls.items():
        torch.cuda.synchronize()
        hip.hipGetLastError()          # start clean
        fn()
        assert hip.hipDeviceSynchronize() == 0, name
        assert hip.hipGetLastError() == 0, name
