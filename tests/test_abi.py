"""The C-ABI library loads, exports every symbol include/ihs.h declares, and
rejects invalid arguments on the host before anything is enqueued (these
calls never reach the GPU, so they run without one)."""
import ctypes
import os
import re

import pytest

import paper_1910_14166_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ihs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ihs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.lib_path()):
        pytest.fail("libihs.so is not built: run __graft_entry__.build()")
    return P.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTS) == names


def test_status_strings(lib):
    assert lib.ihs_status_string(0) == b"ok"
    assert b"positive definite" in lib.ihs_status_string(P.ERR_NOT_PD)
    assert lib.ihs_status_string(99) == b"unknown status"


def dense_struct(n=100, d=8, ld=8, values=1 << 20, batch=1, offs=None):
    s = P.Matrix_t()
    s.format, s.dtype, s.n, s.d, s.ld = P.DENSE, P.F64, n, d, ld
    s.values = values
    s.batch = batch
    s.row_offsets = ctypes.cast(offs, ctypes.c_void_p).value if offs is not None else 0
    return s


def test_invalid_sketch_arguments(lib):
    A = dense_struct()
    ws = ctypes.c_void_p(1 << 20)
    for kind, s, m in [(P.COUNTSKETCH, 2, 8), (P.SJLT, 3, 10), (P.SJLT, 0, 8),
                       (P.COUNTSKETCH, 1, 0), (7, 1, 8)]:
        sk = P.Sketch_t(kind, s, m, 0, 0)
        code = lib.ihs_sketch_apply(ctypes.byref(sk), ctypes.byref(A), ctypes.c_void_p(1 << 20),
                                    P.F64, 8, ws, 1 << 30, None)
        assert code == P.ERR_INVALID_ARG, (kind, s, m)
    big = P.Sketch_t(P.COUNTSKETCH, 1, 1 << 20, 0, 0)
    code = lib.ihs_sketch_apply(ctypes.byref(big), ctypes.byref(A), ctypes.c_void_p(1 << 20),
                                P.F64, 8, ws, 1 << 30, None)
    assert code == P.ERR_UNSUPPORTED


def test_invalid_matrix_and_workspace(lib):
    sk = P.Sketch_t(P.COUNTSKETCH, 1, 16, 0, 0)
    out = ctypes.c_void_p(1 << 20)
    ws = ctypes.c_void_p(1 << 20)
    bad = [dense_struct(ld=4), dense_struct(d=0), dense_struct(n=-1), dense_struct(values=0),
           dense_struct(batch=2, offs=None)]
    for A in bad:
        assert lib.ihs_sketch_apply(ctypes.byref(sk), ctypes.byref(A), out, P.F64, 8, ws,
                                    1 << 30, None) == P.ERR_INVALID_ARG
    offs = (ctypes.c_int64 * 3)(0, 60, 90)  # last offset != n
    A = dense_struct(batch=2, offs=offs)
    assert lib.ihs_sketch_apply(ctypes.byref(sk), ctypes.byref(A), out, P.F64, 8, ws, 1 << 30,
                                None) == P.ERR_INVALID_ARG
    A = dense_struct()
    assert lib.ihs_sketch_apply(ctypes.byref(sk), ctypes.byref(A), out, P.F64, 4, ws, 1 << 30,
                                None) == P.ERR_INVALID_ARG  # ld_sa < d
    assert lib.ihs_sketch_apply(ctypes.byref(sk), ctypes.byref(A), out, P.F64, 8, ws, 16,
                                None) == P.ERR_WORKSPACE
    wide = dense_struct(d=2048, ld=2048)
    assert lib.ihs_sketch_apply(ctypes.byref(sk), ctypes.byref(wide), out, P.F64, 2048, ws,
                                1 << 30, None) == P.ERR_UNSUPPORTED


def test_workspace_query_grows_with_problem(lib):
    o = P.options(64)
    small = lib.ihs_workspace_size(ctypes.byref(dense_struct(n=1000)), ctypes.byref(o))
    large = lib.ihs_workspace_size(ctypes.byref(dense_struct(n=100000)), ctypes.byref(o))
    assert 0 < small < large
    bad = P.options(63, s=2, kind="sjlt")
    assert lib.ihs_workspace_size(ctypes.byref(dense_struct()), ctypes.byref(bad)) == 0


def test_invalid_solve_options(lib):
    A = dense_struct()
    ws = ctypes.c_void_p(1 << 20)
    x = ctypes.c_void_p(1 << 20)
    rep = P.Report_t()
    for o in [P.options(16, constraint="l1", radius=0.0), P.options(16, max_iter=0),
              P.options(16, gram_in="bfloat16", gram_acc="float64"),
              P.options(16, gram_in="float64", gram_acc="float32")]:
        code = lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, None,
                             ctypes.byref(rep), ws, 1 << 30, None)
        assert code == P.ERR_INVALID_ARG
    o = P.options(16, constraint="l1", radius=1.0)
    assert lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, ctypes.c_void_p(8),
                         ctypes.byref(rep), ws, 1 << 30, None) == P.ERR_INVALID_ARG
    # the fixed-sketch method: an unknown method code, a constraint set, and
    # stored factors are refused before any launch
    o = P.options(16, method=2)
    assert lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, None,
                         ctypes.byref(rep), ws, 1 << 30, None) == P.ERR_INVALID_ARG
    o = P.options(16, constraint="l2", radius=1.0, method="fixed_sketch_cg")
    assert lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, None,
                         ctypes.byref(rep), ws, 1 << 30, None) == P.ERR_UNSUPPORTED
    o = P.options(16, method="fixed_sketch_cg", keep_factors=True)
    assert lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, ctypes.c_void_p(8),
                         ctypes.byref(rep), ws, 1 << 30, None) == P.ERR_UNSUPPORTED


def test_tolerance_stop_validation(lib):
    """The step tolerance must be finite and >= 0, and the fixed-sketch
    method has no tolerance stop; all refused before any launch."""
    A = dense_struct()
    ws = ctypes.c_void_p(1 << 20)
    x = ctypes.c_void_p(1 << 20)
    rep = P.Report_t()
    for tol in (-1e-12, float("nan"), float("inf")):
        o = P.options(16, tol=tol)
        assert lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, None,
                             ctypes.byref(rep), ws, 1 << 30, None) == P.ERR_INVALID_ARG, tol
    o = P.options(16, tol=1e-8, method="fixed_sketch_cg")
    assert lib.ihs_solve(ctypes.byref(A), x, ctypes.byref(o), x, None, None,
                         ctypes.byref(rep), ws, 1 << 30, None) == P.ERR_UNSUPPORTED
    # a positive tolerance needs two more d-vectors per problem of workspace
    base = lib.ihs_workspace_size(ctypes.byref(A), ctypes.byref(P.options(16)))
    with_tol = lib.ihs_workspace_size(ctypes.byref(A), ctypes.byref(P.options(16, tol=1e-8)))
    assert with_tol > base


def test_report_layout(lib):
    """The report struct of the binding has the header's field order and size."""
    assert ctypes.sizeof(P.Report_t) == 40
    assert P.Report_t.qp_unpolished.offset == 32


def test_gram_and_qp_validation(lib):
    p = ctypes.c_void_p(1 << 20)
    assert lib.ihs_gram(p, P.BF16, 64, 8, 8, 1, P.F64, p, p, 1 << 30, None) == P.ERR_INVALID_ARG
    assert lib.ihs_gram(p, P.F64, 64, 8, 4, 1, P.F64, p, p, 1 << 30, None) == P.ERR_INVALID_ARG
    assert lib.ihs_gram(p, P.F64, 64, 8, 8, 1, P.F64, p, p, 8, None) == P.ERR_WORKSPACE
    assert lib.ihs_gram_workspace_size(0, 8, 1, P.F64, P.F64) == 0
    o = P.options(1, constraint="l2", radius=-1.0)
    assert lib.ihs_qp_step(8, 1, p, p, p, p, ctypes.byref(o), p, 1 << 30, None,
                           None) == P.ERR_INVALID_ARG


def test_static_sketch_apply_refuses_oversize_before_launch(lib):
    """The allocation-free sketch apply checks the sort state against its
    fixed scratch array on the host: too large a problem is refused with
    IHS_ERR_WORKSPACE before any launch (so this runs without a GPU)."""
    sk = P.Sketch_t(P.COUNTSKETCH, 1, 4096, 0, 0)
    A = dense_struct(n=1 << 30, d=4, ld=4)
    assert lib.ihs_sketch_apply_static(ctypes.byref(sk), ctypes.byref(A), ctypes.c_void_p(8),
                                       P.F64, 4, None) == P.ERR_WORKSPACE
    assert lib.ihs_sketch_apply_static(ctypes.byref(sk), ctypes.byref(A), None, P.F64, 4,
                                       None) == P.ERR_INVALID_ARG


def test_read_ceiling_validation(lib):
    ms = ctypes.c_double()
    assert lib.ihs_profile_read_ceiling(None, 1 << 20, 1, ctypes.byref(ms), None) == \
        P.ERR_INVALID_ARG
    assert lib.ihs_profile_read_ceiling(ctypes.c_void_p(1 << 20), 8, 1, ctypes.byref(ms),
                                        None) == P.ERR_INVALID_ARG
    assert lib.ihs_profile_read_ceiling(ctypes.c_void_p((1 << 20) + 8), 1 << 20, 1,
                                        ctypes.byref(ms), None) == P.ERR_INVALID_ARG


def test_hash_validation(lib):
    sk = P.Sketch_t(P.SJLT, 4, 10, 0, 0)   # 4 does not divide 10
    assert lib.ihs_sketch_hash(ctypes.byref(sk), 10, 0, ctypes.c_void_p(8), ctypes.c_void_p(8),
                               None) == P.ERR_INVALID_ARG
    sk = P.Sketch_t(P.COUNTSKETCH, 1, 10, 0, 0)
    assert lib.ihs_sketch_hash(ctypes.byref(sk), -1, 0, ctypes.c_void_p(8), ctypes.c_void_p(8),
                               None) == P.ERR_INVALID_ARG


def test_last_hip_error_before_any_failure(lib):
    """Host only: with no failed HIP call on this thread the query names
    hipSuccess and writes code 0."""
    code = ctypes.c_int32(-1)
    assert lib.ihs_last_hip_error(ctypes.byref(code)) == b"hipSuccess"
    assert code.value == 0
    assert lib.ihs_last_hip_error(None) == b"hipSuccess"


def test_inverse_threshold_stated_once():
    """The width from which the steps apply an explicit inverse is one
    constant in the HIP sources, and the tests' copy of it matches."""
    from conftest import INVERSE_MIN_D
    csrc = os.path.join(ROOT, "paper_1910_14166_amd", "csrc")
    defs = []
    for name in os.listdir(csrc):
        text = open(os.path.join(csrc, name)).read()
        defs += re.findall(r"constexpr\s+int64_t\s+\w*InverseMinD\s*=\s*(\d+)\s*;", text)
    assert defs == [str(INVERSE_MIN_D)]
