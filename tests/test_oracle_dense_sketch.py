"""Pins of the dense-sketch oracle (SRHT and Gaussian, Sec. 2) to things
other than itself: scipy's Sylvester Hadamard matrix, integer data (exact in
any order), the exact unit diagonal of S^T S for the SRHT, E[S^T S] = I with
the closed-form variance of its entries, the normal distribution of the
Box-Muller entries, and closed forms of the sketch error of Fig. 2."""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.linalg import hadamard

from oracle import dense_sketch as DS
from oracle import philox as PH


@pytest.mark.parametrize("N", [1, 2, 8, 64, 256])
def test_fwht_is_the_sylvester_hadamard_product(N):
    g = np.random.default_rng(N)
    Y = g.integers(-50, 50, size=(N, 3)).astype(np.float64)
    assert np.array_equal(DS.fwht(Y), hadamard(N).astype(np.float64) @ Y)


def test_padded_length():
    assert [DS.padded_rows(n) for n in (0, 1, 2, 3, 4, 5, 1000, 1024, 1025)] == \
        [1, 1, 2, 4, 4, 8, 1024, 1024, 2048]


@pytest.mark.parametrize("n,m", [(5, 3), (8, 8), (37, 20), (128, 500)])
def test_srht_apply_equals_explicit_product(n, m):
    """S built entry by entry from the Sylvester matrix, the sampled rows and
    the signs: on integer data the unscaled product is exact in any order."""
    g = np.random.default_rng(n + m)
    A = g.integers(-20, 20, size=(n, 4)).astype(np.float64)
    N = DS.padded_rows(n)
    rows = DS.srht_rows(9, 2, m, N)
    sg = DS.srht_signs(9, 2, n)
    Hn = hadamard(N).astype(np.float64)
    S_unscaled = np.array([[Hn[rows[k], i] * sg[i] for i in range(n)] for k in range(m)])
    want = (S_unscaled @ A) * (1.0 / math.sqrt(m))
    assert np.array_equal(DS.sketch_apply_srht(A, 9, 2, m), want)
    # and the explicit matrix of the oracle is the same S
    np.testing.assert_allclose(DS.dense_srht_matrix(9, 2, n, m) * math.sqrt(m), S_unscaled,
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [48, 64])
def test_srht_gram_diagonal_is_exactly_one(n):
    """(S^T S)_ii = (1/m) sum_k H[p_k, i]^2 D_i^2 = 1 for every draw."""
    for seed in range(5):
        S = DS.dense_srht_matrix(seed, 0, n, 32)
        np.testing.assert_allclose(np.diag(S.T @ S), 1.0, rtol=0, atol=1e-14)


def test_srht_rows_uniform_and_signs_balanced():
    N, m = 64, 200000
    rows = DS.srht_rows(3, 1, m, N)
    assert rows.min() >= 0 and rows.max() < N
    counts = np.bincount(rows, minlength=N)
    chi2 = ((counts - m / N) ** 2 / (m / N)).sum()
    assert stats.chi2.sf(chi2, N - 1) > 1e-4
    sg = DS.srht_signs(3, 1, m)
    assert abs(sg.sum()) < 5 * math.sqrt(m)


def test_gaussian_entries_are_standard_normal():
    G = DS.gaussian_matrix(7, 4, 8, 50000)
    z = G.ravel()
    assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(z.mean()) < 5 / math.sqrt(len(z))
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / len(z))
    # rows 4q .. 4q+3 of one column come from one Philox call: entry (5, 11)
    # by hand from the scalar generator
    w = PH.philox4x64_scalar((11, 1, 0, DS.STREAM_GAUSSIAN), (7, 4))
    u1 = ((w[0] >> 11) + 1) / 2.0 ** 53
    u2 = (w[1] >> 11) / 2.0 ** 53
    want = math.sqrt(-2.0 * math.log(u1)) * math.sin(2.0 * math.pi * u2)
    assert abs(G[5, 11] - want) <= 4e-16 * max(1.0, abs(want))


@pytest.mark.parametrize("kind", ["srht", "gaussian"])
def test_unbiased_gram_closed_form_variance(kind):
    """E[S^T S] = I. Off-diagonal entries have variance 1/m for both sketches
    (sums of m independent +-1/m, or of m products of independent normals
    over m); Gaussian diagonal entries 2/m. The mean over K draws is tested
    by z-scores."""
    n, m, K = 24, 16, 600
    acc = np.zeros((n, n))
    for seed in range(K):
        S = (DS.dense_srht_matrix(seed, 1, n, m) if kind == "srht"
             else DS.dense_gaussian_matrix(seed, 1, n, m))
        acc += S.T @ S
    mean = acc / K
    off = ~np.eye(n, dtype=bool)
    z_off = (mean[off]) / math.sqrt(1.0 / (m * K))
    assert np.abs(z_off).max() < 5.0
    if kind == "gaussian":
        z_diag = (np.diag(mean) - 1.0) / math.sqrt(2.0 / (m * K))
        assert np.abs(z_diag).max() < 5.0


def test_gaussian_sketch_error_closed_form():
    """E ||A^T S^T S A - A^T A||_F^2 = (||A||_F^4 + ||A^T A||_F^2) / m for the
    Gaussian sketch (a_k = A^T g_k ~ N(0, A^T A): E||a||^4 = (tr M)^2 +
    2 ||M||_F^2). Mean over 300 seeds against it."""
    g = np.random.default_rng(5)
    A = g.standard_normal((40, 5)) * np.array([1.0, 2.0, 0.5, 3.0, 1.0])
    M = A.T @ A
    m = 20
    want = (np.linalg.norm(A) ** 4 + np.linalg.norm(M) ** 2) / m
    errs = np.array([np.linalg.norm(DS.sketch_apply_gaussian(A, s, 0, m).T
                                    @ DS.sketch_apply_gaussian(A, s, 0, m) - M) ** 2
                     for s in range(300)])
    assert abs(errs.mean() - want) < 5 * errs.std() / math.sqrt(len(errs))


def test_srht_sketch_error_conditional_closed_form():
    """Given D, the rows of P are independent uniform draws from the rows y_r
    of H D A, so E[||A^T S^T S A - A^T A||_F^2 | D]
      = (1/m) ((1/N) sum_r ||y_r||^4 - ||A^T A||_F^2).
    The residuals (observed - conditional expectation) over 400 seeds have
    mean zero."""
    g = np.random.default_rng(6)
    A = g.standard_normal((50, 4))
    M = A.T @ A
    n, m = A.shape[0], 16
    N = DS.padded_rows(n)
    res = []
    for s in range(400):
        Y = np.zeros((N, 4))
        Y[:n] = DS.srht_signs(s, 0, n)[:, None] * A
        Y = DS.fwht(Y)
        cond = ((np.sum(Y ** 2, axis=1) ** 2).mean() - np.linalg.norm(M) ** 2) / m
        SA = DS.sketch_apply_srht(A, s, 0, m)
        res.append(np.linalg.norm(SA.T @ SA - M) ** 2 - cond)
    res = np.array(res)
    assert abs(res.mean()) < 5 * res.std() / math.sqrt(len(res))


def test_streams_differ_from_the_sparse_embedding():
    """The SRHT signs and the CountSketch signs of one key are different
    draws (stream word 1 against 0)."""
    from oracle import sketch as OS
    _, cs = OS.sketch_hash(3, 0, 4096, 64)
    sr = DS.srht_signs(3, 0, 4096)
    assert np.mean(cs[:, 0] == sr) < 0.55
