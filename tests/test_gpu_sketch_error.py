"""The empirical sketch error of App. B, Fig. 2, through the library:
err(S) = ||A^T S^T S A - A^T A||_F / ||A^T A||_F for CountSketch and the SJLT
on a W8A-shaped sparse matrix (49749 x 300, 4% dense, binary values).

Two bars. (1) Parity: with binary A every entry of S A is an integer (a
multiple of 1/2 for the SJLT with s = 4) and every entry of H = (SA)^T SA is
exact in float64 in any summation order, so the library's H equals the
oracle's H bit for bit. (2) The expectation: over K seeds the mean of
err^2 ||A^T A||_F^2 matches the closed form
E ||A^T S^T S A - A^T A||_F^2 = (||A||_F^4 + ||A^T A||_F^2 - 2 sum_i ||a_i||^4) / m
(a consequence of E[S^T S] = I and the independence of the hash, Lemma A.7)
within five standard errors."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ihs as O
from oracle import sketch as OS

pytestmark = pytest.mark.gpu


def closed_form(indptr, indices, data, n, d):
    """Expected squared Frobenius error times m, and ||A^T A||_F, from plain
    float64 sums over the CSR arrays."""
    import scipy.sparse as sp
    A = sp.csr_matrix((data, indices, indptr), shape=(n, d))
    AtA = (A.T @ A).toarray()
    rn = np.asarray(A.multiply(A).sum(axis=1)).ravel()
    fro2 = rn.sum()
    return fro2 ** 2 + (AtA ** 2).sum() - 2 * (rn ** 2).sum(), AtA


@pytest.fixture(scope="module")
def w8a(gpu_lib):
    import torch
    wl = W.table1_like("w8a")
    M = gpu_lib.Matrix(row_ptr=torch.from_numpy(wl.indptr).cuda(),
                       col_idx=torch.from_numpy(wl.indices).cuda(),
                       values=torch.from_numpy(wl.data).cuda(), n=wl.n, d=wl.d)
    return wl, M


@pytest.mark.parametrize("kind,s,m", [("countsketch", 1, 600), ("sjlt", 4, 600),
                                      ("countsketch", 1, 3000), ("sjlt", 4, 3000)])
def test_sketched_gram_bit_exact_on_binary_data(gpu_lib, w8a, kind, s, m):
    P = gpu_lib
    wl, M = w8a
    spec = P.SketchSpec(m, s, kind, seed=77, iter=1)
    SA = P.sketch_apply(M, spec)
    H = P.gram(SA, m).cpu().numpy()[0]
    ref_SA = OS.sketch_apply_csr(wl.indptr, wl.indices, wl.data, wl.n, wl.d, 77, 1, m, s)
    assert np.array_equal(SA.cpu().numpy(), ref_SA)
    assert np.array_equal(H, O.gram(ref_SA))


@pytest.mark.parametrize("kind,s,m", [("countsketch", 1, 600), ("sjlt", 4, 1500)])
def test_mean_sketch_error_matches_closed_form(gpu_lib, w8a, kind, s, m):
    import torch
    P = gpu_lib
    wl, M = w8a
    pred_m, AtA = closed_form(wl.indptr, wl.indices, wl.data, wl.n, wl.d)
    AtA_dev = torch.from_numpy(AtA).cuda()
    K = 40
    vals = np.empty(K)
    for seed in range(K):
        SA = P.sketch_apply(M, P.SketchSpec(m, s, kind, seed=1000 + seed, iter=0))
        H = P.gram(SA, m)[0]
        vals[seed] = float(((H - AtA_dev) ** 2).sum())
    pred = pred_m / m
    se = vals.std(ddof=1) / math.sqrt(K)
    assert abs(vals.mean() - pred) < 5 * se, (vals.mean(), pred, se)
    # the normalised error of Fig. 2 is about sqrt(pred) / ||A^T A||_F
    rel = np.sqrt(vals) / np.linalg.norm(AtA)
    assert 0.5 < rel.mean() / (math.sqrt(pred) / np.linalg.norm(AtA)) < 1.5
