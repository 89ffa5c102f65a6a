"""Python binding of libihs, the MI355X (gfx950) Iterative Hessian Sketch library.

Every function marshals torch tensors (device memory) into the C ABI of
include/ihs.h and calls it on the current HIP stream. All arithmetic runs in
the library's HIP kernels; nothing here computes a result. The library must be
built (`python -m paper_1910_14166_amd.build`); importing works without it,
but load() and every call raise RuntimeError while libihs.so is missing, and
a failing library call raises IHSError (for IHS_ERR_HIP with the HIP error
behind it).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libihs.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_NOT_PD, \
    ERR_NOT_CONVERGED, ERR_NONFINITE = range(8)
F64, F32, BF16 = 0, 1, 2
COUNTSKETCH, SJLT, SRHT, GAUSSIAN = 0, 1, 2, 3
_KINDS = {"countsketch": COUNTSKETCH, "sjlt": SJLT, "srht": SRHT, "gaussian": GAUSSIAN}
UNCONSTRAINED, L1_BALL, L2_BALL, L1_PENALTY = 0, 1, 2, 3
DENSE, CSR = 0, 1
METHOD_IHS, METHOD_FIXED_SKETCH_CG = 0, 1

_CONSTRAINTS = {"none": UNCONSTRAINED, "l1": L1_BALL, "l2": L2_BALL, "l1_penalty": L1_PENALTY}
_DTYPES = {"float64": F64, "float32": F32, "bfloat16": BF16,
           "f64": F64, "f32": F32, "bf16": BF16}

EXPORTS = ["ihs_status_string", "ihs_last_hip_error", "ihs_sketch_hash", "ihs_workspace_size",
           "ihs_sketch_apply", "ihs_sketch_apply_static", "ihs_sketch_adjoint", "ihs_gram_workspace_size",
           "ihs_gram", "ihs_gradient", "ihs_qp_workspace_size", "ihs_qp_step",
           "ihs_solve", "ihs_adjoint_solve", "ihs_solution_grads",
           "ihs_profile_enable", "ihs_profile_read", "ihs_profile_read_ceiling"]


class IHSError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = _status_text(code)
        super().__init__(f"{where}: {msg} (status {code})" if where else msg)


class Matrix_t(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("values", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("batch", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("row_offsets", ctypes.c_void_p)]


class Sketch_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("s", ctypes.c_int32), ("m", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("iter", ctypes.c_uint64)]


class Options_t(ctypes.Structure):
    _fields_ = [("constraint", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("radius", ctypes.c_double), ("sketch", Sketch_t),
                ("gram_in", ctypes.c_int32), ("gram_acc", ctypes.c_int32),
                ("qp_max_inner", ctypes.c_int32), ("keep_factors", ctypes.c_int32),
                ("qp_tol", ctypes.c_double), ("tol", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("method", ctypes.c_int32)]


class Report_t(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("failed_iter", ctypes.c_int32), ("failed_problem", ctypes.c_int32),
                ("objective", ctypes.c_double), ("last_step", ctypes.c_double),
                ("qp_unpolished", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib_path():
    return LIB_PATH


def load(path: Optional[str] = None):
    """Load libihs.so (raises IHSError-like RuntimeError when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libihs.so not built at {p}; run "
                           "`python -m paper_1910_14166_amd.build`")
    L = ctypes.CDLL(p)
    vp, i32, i64, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint64, ctypes.c_size_t)
    M, S, O, R = (ctypes.POINTER(Matrix_t), ctypes.POINTER(Sketch_t),
                  ctypes.POINTER(Options_t), ctypes.POINTER(Report_t))
    sig = {
        "ihs_status_string": (ctypes.c_char_p, [i32]),
        "ihs_last_hip_error": (ctypes.c_char_p, [ctypes.POINTER(i32)]),
        "ihs_sketch_hash": (i32, [S, i64, i32, vp, vp, vp]),
        "ihs_workspace_size": (sz, [M, O]),
        "ihs_sketch_apply": (i32, [S, M, vp, i32, i64, vp, sz, vp]),
        "ihs_sketch_apply_static": (i32, [S, M, vp, i32, i64, vp]),
        "ihs_sketch_adjoint": (i32, [S, i64, i64, i32, vp, vp, i64, vp, i64, vp]),
        "ihs_gram_workspace_size": (sz, [i64, i64, i32, i32, i32]),
        "ihs_gram": (i32, [vp, i32, i64, i64, i64, i32, i32, vp, vp, sz, vp]),
        "ihs_gradient": (i32, [M, vp, vp, vp, vp, vp, vp, sz, vp]),
        "ihs_qp_workspace_size": (sz, [i64, i32, O]),
        "ihs_qp_step": (i32, [i64, i32, vp, vp, vp, vp, O, vp, sz, vp, R]),
        "ihs_solve": (i32, [M, vp, O, vp, vp, vp, R, vp, sz, vp]),
        "ihs_adjoint_solve": (i32, [M, vp, vp, i32, vp, vp, sz, vp]),
        "ihs_solution_grads": (i32, [M, vp, vp, vp, vp, vp, i64, vp]),
        "ihs_profile_enable": (None, [i32]),
        "ihs_profile_read": (i32, [ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]),
        "ihs_profile_read_ceiling": (i32, [vp, i64, i32, ctypes.POINTER(ctypes.c_double), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _status_text(code):
    try:
        return load().ihs_status_string(int(code)).decode()
    except Exception:
        return "status %d" % code


def _check(code, where):
    if code == ERR_HIP:
        hc = ctypes.c_int32(0)
        name = load().ihs_last_hip_error(ctypes.byref(hc)).decode()
        raise IHSError(code, "%s (%s, %d)" % (where, name, hc.value))
    if code != OK:
        raise IHSError(code, where)


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dt(x):
    if isinstance(x, int):
        return x
    return _DTYPES[str(x).replace("torch.", "")]


def _torch_dtype(code):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[code]


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class SketchSpec:
    """A sketch of m rows per problem: "countsketch" (s = 1), "sjlt" (s
    blocks), or the dense "srht" and "gaussian" sketches (s = 1)."""
    m: int
    s: int = 1
    kind: str = "countsketch"
    seed: int = 0
    iter: int = 0

    def struct(self):
        kind = _KINDS[self.kind] if isinstance(self.kind, str) else int(self.kind)
        return Sketch_t(kind, int(self.s), int(self.m), int(self.seed) & (2 ** 64 - 1),
                        int(self.iter) & (2 ** 64 - 1))


class Matrix:
    """A (ragged batch of) dense or CSR data matrices on the device."""

    def __init__(self, dense=None, row_ptr=None, col_idx=None, values=None, n=None,
                 d=None, row_offsets=None):
        torch = _torch()
        self.dense, self.row_ptr, self.col_idx, self.values = dense, row_ptr, col_idx, values
        self._offs = None
        if dense is not None:
            assert dense.dim() == 2 and dense.stride(1) == 1
            self.n, self.d = dense.shape
            self.ld = dense.stride(0)
            self.dtype = F64 if dense.dtype == torch.float64 else F32
            self.format = DENSE
        else:
            self.n, self.d, self.ld = int(n), int(d), int(d)
            self.dtype = F64
            self.format = CSR
        self.batch = 1
        if row_offsets is not None:
            offs = [int(v) for v in row_offsets]
            self.batch = len(offs) - 1
            self._offs = (ctypes.c_int64 * len(offs))(*offs)
        self.row_offsets = None if self._offs is None else list(self._offs)
        self._s = Matrix_t()
        s = self._s
        s.format, s.dtype, s.n, s.d, s.ld = self.format, self.dtype, self.n, self.d, self.ld
        if self.format == DENSE:
            s.values = dense.data_ptr()
        else:
            s.values, s.row_ptr, s.col_idx = values.data_ptr(), row_ptr.data_ptr(), \
                col_idx.data_ptr() if col_idx.numel() else 0
            s.nnz = values.numel()
        s.batch = self.batch
        s.row_offsets = ctypes.cast(self._offs, ctypes.c_void_p).value if self._offs else 0

    @property
    def device(self):
        return (self.dense if self.dense is not None else self.row_ptr).device

    def ref(self):
        return ctypes.byref(self._s)


def options(m, s=1, kind="countsketch", seed=0, iter0=0, max_iter=10, constraint="none",
            radius=0.0, gram_in="float64", gram_acc="float64", keep_factors=False,
            qp_max_inner=0, qp_tol=0.0, tol=0.0, schedule="overlap", method="ihs"):
    o = Options_t()
    o.constraint = _CONSTRAINTS[constraint] if isinstance(constraint, str) else constraint
    o.max_iter = int(max_iter)
    o.radius = float(radius)
    o.sketch = SketchSpec(m, s, kind, seed, iter0).struct()
    o.gram_in, o.gram_acc = _dt(gram_in), _dt(gram_acc)
    o.qp_max_inner, o.keep_factors = int(qp_max_inner), int(bool(keep_factors))
    o.qp_tol, o.tol = float(qp_tol), float(tol)
    o.schedule = {"overlap": 0, "sequential": 1, "overlap2": 2}[schedule] \
        if isinstance(schedule, str) \
        else int(schedule)
    o.method = {"ihs": METHOD_IHS, "fixed_sketch_cg": METHOD_FIXED_SKETCH_CG}[method] \
        if isinstance(method, str) else int(method)
    return o


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------
def sketch_hash(n, sketch: SketchSpec, problem=0, device="cuda"):
    torch = _torch()
    L = load()
    bucket = torch.empty(max(n * sketch.s, 1), dtype=torch.int32, device=device)
    sign = torch.empty(max(n * sketch.s, 1), dtype=torch.int8, device=device)
    sk = sketch.struct()
    _check(L.ihs_sketch_hash(ctypes.byref(sk), n, problem, _ptr(bucket), _ptr(sign),
                             _stream()), "ihs_sketch_hash")
    return bucket[: n * sketch.s].view(n, sketch.s), sign[: n * sketch.s].view(n, sketch.s)


def workspace_size(A: Matrix, opts):
    return int(load().ihs_workspace_size(A.ref(), ctypes.byref(opts)))


def sketch_apply(A: Matrix, sketch: SketchSpec, out_dtype="float64", out=None, ws=None):
    torch = _torch()
    L = load()
    dt = _dt(out_dtype)
    if out is None:
        out = torch.empty(A.batch * sketch.m, A.d, dtype=_torch_dtype(dt), device=A.device)
    opts = options(sketch.m, sketch.s, sketch.kind, sketch.seed, sketch.iter)
    need = workspace_size(A, opts)
    if need == 0:
        raise IHSError(ERR_INVALID_ARG, "ihs_workspace_size")
    if ws is None:
        ws = _workspace(need, A.device)
    sk = sketch.struct()
    _check(L.ihs_sketch_apply(ctypes.byref(sk), A.ref(), _ptr(out), dt, out.stride(0),
                              _ptr(ws), ws.numel(), _stream()), "ihs_sketch_apply")
    return out


def sketch_apply_static(A: Matrix, sketch: SketchSpec, out_dtype="float64", out=None):
    """SA through the allocation-free entry point (its sort state lives in the
    library's per-GPU scratch array; calls on one GPU must not overlap). The
    library allocates nothing; pass `out` to allocate nothing here either."""
    torch = _torch()
    L = load()
    dt = _dt(out_dtype)
    if out is None:
        out = torch.empty(A.batch * sketch.m, A.d, dtype=_torch_dtype(dt), device=A.device)
    sk = sketch.struct()
    _check(L.ihs_sketch_apply_static(ctypes.byref(sk), A.ref(), _ptr(out), dt, out.stride(0),
                                     _stream()), "ihs_sketch_apply_static")
    return out


def sketch_adjoint(G, n, sketch: SketchSpec, row_offsets=None, out=None):
    torch = _torch()
    L = load()
    d = G.shape[1]
    if out is None:
        out = torch.empty(n, d, dtype=torch.float64, device=G.device)
    batch = 1 if row_offsets is None else len(row_offsets) - 1
    offs = None if row_offsets is None else (ctypes.c_int64 * (batch + 1))(*[int(v) for v in row_offsets])
    sk = sketch.struct()
    _check(L.ihs_sketch_adjoint(ctypes.byref(sk), n, d, batch,
                                ctypes.cast(offs, ctypes.c_void_p) if offs else None,
                                _ptr(G), G.stride(0), _ptr(out), out.stride(0), _stream()),
           "ihs_sketch_adjoint")
    return out


def gram(SA, m, batch=1, in_dtype=None, acc_dtype="float64", out=None):
    torch = _torch()
    L = load()
    in_dt = _dt(in_dtype if in_dtype is not None else str(SA.dtype))
    acc = _dt(acc_dtype)
    d = SA.shape[1]
    if out is None:
        out = torch.empty(batch, d, d, dtype=torch.float64, device=SA.device)
    need = L.ihs_gram_workspace_size(m, d, batch, in_dt, acc)
    if need == 0:
        raise IHSError(ERR_INVALID_ARG, "ihs_gram_workspace_size")
    ws = _workspace(need, SA.device)
    _check(L.ihs_gram(_ptr(SA), in_dt, m, d, SA.stride(0), batch, acc, _ptr(out), _ptr(ws),
                      ws.numel(), _stream()), "ihs_gram")
    return out


def gradient(A: Matrix, b, x, want_r=False):
    torch = _torch()
    L = load()
    g = torch.empty(A.batch, A.d, dtype=torch.float64, device=A.device)
    f = torch.empty(A.batch, dtype=torch.float64, device=A.device)
    r = torch.empty(A.n, dtype=torch.float64, device=A.device) if want_r else None
    need = workspace_size(A, options(1))
    ws = _workspace(need, A.device)
    _check(L.ihs_gradient(A.ref(), _ptr(b), _ptr(x), _ptr(g), _ptr(r), _ptr(f), _ptr(ws),
                          ws.numel(), _stream()), "ihs_gradient")
    return g, r, f


def qp_step(H, g, x, constraint="none", radius=0.0, qp_max_inner=0, qp_tol=0.0, out=None,
            want_report=False):
    """x^{t+1} of Eq.(2) for each problem; with want_report, (x^{t+1}, report)."""
    torch = _torch()
    L = load()
    batch, d = g.shape
    if out is None:
        out = torch.empty_like(x)
    o = options(1, constraint=constraint, radius=radius, qp_max_inner=qp_max_inner,
                qp_tol=qp_tol)
    need = L.ihs_qp_workspace_size(d, batch, ctypes.byref(o))
    ws = _workspace(need, g.device)
    rep = Report_t()
    _check(L.ihs_qp_step(d, batch, _ptr(H), _ptr(g), _ptr(x), _ptr(out), ctypes.byref(o),
                         _ptr(ws), ws.numel(), _stream(), ctypes.byref(rep)), "ihs_qp_step")
    return (out, rep) if want_report else out


@dataclass
class SolveResult:
    x: object
    history: object
    factors: object
    report: Report_t


def solve(A: Matrix, b, opts, x0=None, history=False, factors=False, ws=None,
          raise_on_error=True):
    torch = _torch()
    L = load()
    x = torch.zeros(A.batch, A.d, dtype=torch.float64, device=A.device) if x0 is None \
        else x0.clone()
    hist = torch.empty(opts.max_iter, A.batch, A.d, dtype=torch.float64, device=A.device) \
        if history else None
    fac = torch.empty(opts.max_iter, A.batch, A.d, A.d, dtype=torch.float64,
                      device=A.device) if factors else None
    if factors:
        opts.keep_factors = 1
    need = workspace_size(A, opts)
    if need == 0:
        raise IHSError(ERR_INVALID_ARG, "ihs_workspace_size")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, A.device)
    rep = Report_t()
    code = L.ihs_solve(A.ref(), _ptr(b), ctypes.byref(opts), _ptr(x), _ptr(hist), _ptr(fac),
                       ctypes.byref(rep), _ptr(ws), ws.numel(), _stream())
    if raise_on_error:
        _check(code, "ihs_solve")
    return SolveResult(x, hist, fac, rep)


def adjoint_solve(A: Matrix, xbar, factors):
    torch = _torch()
    L = load()
    lam = torch.empty(A.batch, A.d, dtype=torch.float64, device=A.device)
    need = workspace_size(A, options(1)) + 2 * A.batch * A.d * 8 + 1024
    ws = _workspace(need, A.device)
    _check(L.ihs_adjoint_solve(A.ref(), _ptr(xbar), _ptr(factors), factors.shape[0],
                               _ptr(lam), _ptr(ws), ws.numel(), _stream()),
           "ihs_adjoint_solve")
    return lam


def solution_grads(A: Matrix, b, x, lam, want_db=True, want_dA=True):
    torch = _torch()
    L = load()
    db = torch.empty(A.n, dtype=torch.float64, device=A.device) if want_db else None
    dA = torch.empty(A.n, A.d, dtype=torch.float64, device=A.device) if want_dA else None
    _check(L.ihs_solution_grads(A.ref(), _ptr(b), _ptr(x), _ptr(lam), _ptr(db), _ptr(dA),
                                A.d, _stream()), "ihs_solution_grads")
    return db, dA


def profile_enable(on=True):
    load().ihs_profile_enable(1 if on else 0)


def profile_read():
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().ihs_profile_read(ctypes.byref(n), ctypes.byref(ms)), "ihs_profile_read")
    return int(n.value), float(ms.value)


def read_ceiling(buf, reps=5):
    """GB/s of reading the device tensor `buf` once (the library's read probe)."""
    ms = ctypes.c_double()
    nbytes = buf.numel() * buf.element_size() // 16 * 16
    _check(load().ihs_profile_read_ceiling(_ptr(buf), nbytes, int(reps), ctypes.byref(ms),
                                           _stream()), "ihs_profile_read_ceiling")
    return nbytes / (ms.value * 1e-3) / 1e9
