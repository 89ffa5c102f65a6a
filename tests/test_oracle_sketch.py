"""Pins for the oracle's sketch application and adjoint: an explicit dense S
(Sec. 2 definitions), integer data (every summation order exact), math.fsum,
Lemmas A.5-A.7 and the closed-form variance of (SA)^T SA."""
import math

import numpy as np
import pytest

from oracle.sketch import (dense_sketch_matrix, round_to_bf16, sketch_adjoint,
                           sketch_apply_csr, sketch_apply_dense, sketch_hash)
from workloads import csr_to_dense


@pytest.mark.parametrize("n,d,m,s", [(37, 5, 8, 1), (200, 3, 16, 4),
                                     (5, 7, 64, 1), (300, 9, 12, 4), (1, 1, 4, 1)])
def test_dense_apply_equals_explicit_S_on_integers(n, d, m, s):
    g = np.random.default_rng(n + d)
    A = g.integers(-1000, 1000, size=(n, d)).astype(np.float64)
    S = dense_sketch_matrix(3, 5, n, m, s)
    assert np.array_equal(sketch_apply_dense(A, 3, 5, m, s), S @ A)


def test_dense_apply_s2_scaled_after_sum():
    g = np.random.default_rng(1)
    A = g.integers(-50, 50, size=(90, 4)).astype(np.float64)
    S = dense_sketch_matrix(0, 1, 90, 10, 2)
    # S carries +-1/sqrt(2); the library scales the exact integer sum once
    ref = np.round(S @ A * math.sqrt(2)) / math.sqrt(2)
    assert np.allclose(sketch_apply_dense(A, 0, 1, 10, 2), ref, rtol=0, atol=1e-12)
    exact_sum = np.round(S * math.sqrt(2)) @ A
    assert np.array_equal(sketch_apply_dense(A, 0, 1, 10, 2),
                          exact_sum * (1.0 / math.sqrt(2)))


def test_dense_apply_matches_sequential_fsum_bound():
    g = np.random.default_rng(2)
    n, d, m = 400, 6, 8
    A = g.standard_normal((n, d))
    SA = sketch_apply_dense(A, 9, 0, m, 1)
    bucket, sign = sketch_hash(9, 0, n, m, 1)
    u = 2.0 ** -53
    for r in range(m):
        rows = np.nonzero(bucket[:, 0] == r)[0]
        for j in range(d):
            terms = [sign[i, 0] * A[i, j] for i in rows]
            exact = math.fsum(terms)
            bound = len(terms) * u * sum(abs(t) for t in terms) + 1e-300
            assert abs(SA[r, j] - exact) <= bound
            seq = 0.0
            for t in terms:
                seq += t
            assert SA[r, j] == seq


def test_csr_apply_equals_dense_apply_bitwise():
    g = np.random.default_rng(3)
    n, d = 500, 20
    dense = g.standard_normal((n, d)) * (g.random((n, d)) < 0.15)
    dense[7] = 0.0
    indptr = np.zeros(n + 1, dtype=np.int64)
    indptr[1:] = np.cumsum((dense != 0).sum(1))
    rows, cols = np.nonzero(dense)
    for s in (1, 4):
        a = sketch_apply_csr(indptr, cols, dense[rows, cols], n, d, 4, 2, 32, s)
        b = sketch_apply_dense(dense, 4, 2, 32, s)
        assert np.array_equal(a, b)
    assert np.array_equal(csr_to_dense(indptr, cols, dense[rows, cols], n, d), dense)


def test_csr_apply_explicit_S_integers():
    g = np.random.default_rng(4)
    n, d, m = 120, 10, 16
    dense = g.integers(-9, 9, size=(n, d)).astype(float) * (g.random((n, d)) < 0.3)
    indptr = np.zeros(n + 1, dtype=np.int64)
    indptr[1:] = np.cumsum((dense != 0).sum(1))
    rows, cols = np.nonzero(dense)
    S = dense_sketch_matrix(1, 1, n, m, 4)
    assert np.array_equal(
        sketch_apply_csr(indptr, cols, dense[rows, cols], n, d, 1, 1, m, 4), S @ dense)


def test_reduced_precision_outputs():
    g = np.random.default_rng(5)
    A = g.standard_normal((64, 8))
    sa64 = sketch_apply_dense(A, 0, 0, 16, 1)
    assert np.array_equal(sketch_apply_dense(A, 0, 0, 16, 1, out_dtype="float32"),
                          sa64.astype(np.float32))
    bf = sketch_apply_dense(A, 0, 0, 16, 1, out_dtype="bfloat16")
    assert np.all(np.abs(bf - sa64) <= np.abs(sa64) * 2.0 ** -8)


def test_bf16_rounding_against_torch_on_float32_values():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(6)
    x32 = (g.standard_normal(20000) * 10.0 ** g.integers(-5, 5, 20000)).astype(np.float32)
    # exact ties: bf16 value + half an ulp
    base = torch.tensor(x32[:1000]).to(torch.bfloat16).float().numpy()
    ulp = np.abs(base) * 0 + 2.0 ** (np.floor(np.log2(np.abs(base))) - 7)
    x32[:1000] = (base + 0.5 * ulp).astype(np.float32)
    ref = torch.tensor(x32).to(torch.bfloat16).double().numpy()
    ours = round_to_bf16(x32.astype(np.float64))
    assert np.array_equal(ours, ref)


def test_lemma_a5_rows_orthogonal_counts_on_diagonal():
    n, m = 500, 23
    S = dense_sketch_matrix(12, 3, n, m, 1)
    SSt = S @ S.T
    bucket, _ = sketch_hash(12, 3, n, m, 1)
    counts = np.bincount(bucket[:, 0], minlength=m)
    assert np.array_equal(SSt, np.diag(counts.astype(float)))


def test_lemma_a6_expected_SSt():
    n, m, K = 200, 10, 400
    diag = np.zeros(m)
    for seed in range(K):
        bucket, _ = sketch_hash(seed, 0, n, m, 1)
        diag += np.bincount(bucket[:, 0], minlength=m)
    mean = diag / K
    sd = math.sqrt(n * (1 / m) * (1 - 1 / m) / K)
    assert np.all(np.abs(mean - n / m) < 5 * sd)


@pytest.mark.parametrize("s", [1, 4])
def test_lemma_a7_expected_StS_identity(s):
    n, m, K = 6, 8, 3000
    acc = np.zeros((n, n))
    for seed in range(K):
        S = dense_sketch_matrix(seed, 1, n, m, s)
        acc += S.T @ S
    mean = acc / K
    assert np.allclose(np.diag(mean), 1.0, atol=1e-12)
    off = mean[~np.eye(n, dtype=bool)]
    assert np.all(np.abs(off) < 5 * math.sqrt(1.0 / m / K))


@pytest.mark.parametrize("s", [1, 4])
def test_unbiased_gram_with_closed_form_variance(s):
    g = np.random.default_rng(7)
    n, d, m, K = 60, 3, 16, 1500
    A = g.standard_normal((n, d))
    AtA = A.T @ A
    acc = np.zeros((d, d))
    for seed in range(K):
        SA = sketch_apply_dense(A, seed, 0, m, s)
        acc += SA.T @ SA
    mean = acc / K
    # Var[(SA)^T SA]_jk = (1/m) sum_{i != l} (A_ij^2 A_lk^2 + A_ij A_ik A_lj A_lk)
    var = np.zeros((d, d))
    for j in range(d):
        for k in range(d):
            a2 = A[:, j] ** 2
            b2 = A[:, k] ** 2
            p = A[:, j] * A[:, k]
            var[j, k] = (a2.sum() * b2.sum() - (a2 * b2).sum()
                         + p.sum() ** 2 - (p * p).sum()) / m
    z = (mean - AtA) / np.sqrt(var / K)
    assert np.all(np.abs(z) < 5.0)


@pytest.mark.parametrize("s", [1, 4])
def test_frobenius_error_closed_form(s):
    """E ||A^T S^T S A - A^T A||_F^2 = (||A||_F^4 + ||A^T A||_F^2 - 2 sum_i ||a_i||^4)/m,
    the expectation behind the empirical sketch-error metric of App. B."""
    g = np.random.default_rng(8)
    n, d, m, K = 80, 4, 32, 3000
    A = g.standard_normal((n, d))
    AtA = A.T @ A
    rn = (A ** 2).sum(1)
    pred = ((A ** 2).sum() ** 2 + (AtA ** 2).sum() - 2 * (rn ** 2).sum()) / m
    vals = np.empty(K)
    for seed in range(K):
        SA = sketch_apply_dense(A, seed, 2, m, s)
        vals[seed] = ((SA.T @ SA - AtA) ** 2).sum()
    se = vals.std() / math.sqrt(K)
    assert abs(vals.mean() - pred) < 5 * se


def test_collision_free_sketch_preserves_gram():
    g = np.random.default_rng(9)
    n, d, m = 12, 4, 1 << 22
    A = g.standard_normal((n, d))
    bucket, _ = sketch_hash(2, 0, n, m, 1)
    assert len(np.unique(bucket)) == n
    SA = sketch_apply_dense(A, 2, 0, m, 1)
    assert np.allclose(SA.T @ SA, A.T @ A, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("s", [1, 4])
def test_adjoint_dot_identity_and_explicit(s):
    g = np.random.default_rng(10)
    n, d, m = 70, 5, 16
    X = g.standard_normal((n, d))
    G = g.standard_normal((m, d))
    lhs = np.sum(sketch_apply_dense(X, 6, 1, m, s) * G)
    rhs = np.sum(X * sketch_adjoint(G, n, 6, 1, m, s))
    assert abs(lhs - rhs) < 1e-12 * (np.abs(X).sum() * np.abs(G).max())
    Gi = g.integers(-20, 20, size=(m, d)).astype(float)
    S = dense_sketch_matrix(6, 1, n, m, s)
    assert np.array_equal(sketch_adjoint(Gi, n, 6, 1, m, s), S.T @ Gi)


def test_table1_like_shapes_and_values():
    """The Table 1 stand-ins have the table's shape and density, canonical CSR
    (sorted distinct columns per row) and the stated values."""
    import json
    import os
    import workloads as W
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "table1_datasets.json")))
    for ds in gold["datasets"]:
        if ds["name"] == "W8A" or ds["name"] == "Abtaha":
            wl = W.table1_like(ds["name"])
            assert (wl.n, wl.d) == (ds["n"], ds["d"])
            assert wl.indptr[-1] == round(ds["density"] * ds["n"] * ds["d"])
            for r in range(0, wl.n, 997):
                cols = wl.indices[wl.indptr[r]:wl.indptr[r + 1]]
                assert np.all(np.diff(cols) > 0)
            if ds["name"] == "W8A":
                assert np.all(wl.data == 1.0)
            else:
                assert abs(wl.data.mean()) < 0.01 and abs(wl.data.std() - 1) < 0.01
