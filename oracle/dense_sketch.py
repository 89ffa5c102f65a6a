"""Oracle: the two dense sketches of Sec. 2 ("Sketching Results") that the
paper compares the sparse embeddings with, and their application to A.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Gaussian sketch (Sec. 2): S = G / sqrt(m) with G (m x n) of i.i.d. N(0, 1)
entries. Applying it is a dense product, O(m n d) ("Time Complexity of
sketching methods").

SRHT (Sec. 2; Ailon and Chazelle): S = P H D with D a diagonal of i.i.d.
+-1 signs, H the recursively defined (Sylvester) Hadamard transform and P a
matrix that samples rows uniformly at random. Applying it costs a fast
Hadamard transform plus O(n) for P and D.

Readings of the parts the paper leaves open (both sides take them):
  * H acts on N = 2^ceil(log2 n) rows: A is padded with zero rows, so S is
    the first n columns of the N-point transform. (The experiments of Sec. 3
    instead keep 2^floor(log2 n) of the rows; a caller reproduces that by
    passing the chosen rows as A.)
  * H has entries +-1 (unnormalised) and P draws each of its m rows
    independently and uniformly from the N rows (with replacement); the scale
    1/sqrt(m) makes E[S^T S] = I, the normalisation the paper's embeddings
    share (App. A.1.1, Lemma A.7 for the sparse ones).
  * The transform is the radix-2 one in the order of the recursion: stages
    h = 1, 2, 4, ..., N/2, each replacing the pair (y_i, y_{i+h}) (bit h of i
    clear) by (y_i + y_{i+h}, y_i - y_{i+h}). The scale is applied once, to
    the sampled rows.
  * The Gram-side scale 1/sqrt(m) of the Gaussian sketch is applied once,
    after the product G A.

Random choices, drawn from Philox4x64-10 under key (seed, iteration) like the
sparse embeddings, on counter words (., ., problem, stream) with a stream
word of their own (0 belongs to the sparse embeddings):
  stream 1, counter (i, 0, p, 1):  D_i = -1 if bit 63 of word 1 is set, else +1
  stream 2, counter (k, 0, p, 2):  row k of P samples row floor(word 0 * N / 2^64)
  stream 3, counter (i, q, p, 3):  G[4q + j, i], j = 0..3, by the Box-Muller
        method (Box and Muller, 1958) from words (0, 1) and (2, 3):
        u1 = ((w_a >> 11) + 1) / 2^53 in (0, 1],  u2 = (w_b >> 11) / 2^53,
        rho = sqrt(-2 ln u1),  G[4q + 2h] = rho cos(2 pi u2),
        G[4q + 2h + 1] = rho sin(2 pi u2)   for (a, b) = (0, 1), (2, 3)
"""
from __future__ import annotations

import math

import numpy as np

from .philox import mulhilo64, philox4x64
from .sketch import round_output

STREAM_SRHT_SIGN = 1
STREAM_SRHT_ROWS = 2
STREAM_GAUSSIAN = 3


def padded_rows(n):
    """N = 2^ceil(log2 n): the length the Hadamard transform acts on."""
    return 1 if n <= 1 else 1 << (int(n) - 1).bit_length()


# --------------------------------------------------------------------------
# SRHT
# --------------------------------------------------------------------------
def srht_signs(seed, iteration, n, problem=0):
    """The diagonal of D: +-1 per row, as float64."""
    w = philox4x64(np.arange(n, dtype=np.uint64), 0, problem, STREAM_SRHT_SIGN, seed, iteration)
    return np.where((w[1] >> np.uint64(63)) != 0, -1.0, 1.0)


def srht_rows(seed, iteration, m, N, problem=0):
    """The m rows of the N-point transform that P samples (with replacement)."""
    w = philox4x64(np.arange(m, dtype=np.uint64), 0, problem, STREAM_SRHT_ROWS, seed, iteration)
    hi, _ = mulhilo64(w[0], np.uint64(N))
    return hi.astype(np.int64)


def fwht(Y):
    """Unnormalised Walsh-Hadamard transform of the rows of Y (N = len(Y), a
    power of two), radix 2 in the order of the recursion: H_N Y with H_N the
    Sylvester matrix [[H, H], [H, -H]]."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    N = Y.shape[0]
    h = 1
    while h < N:
        Y = Y.reshape(N // (2 * h), 2, h, *Y.shape[1:])
        a = Y[:, 0].copy()
        b = Y[:, 1].copy()
        Y[:, 0] = a + b
        Y[:, 1] = a - b
        Y = Y.reshape(N, *Y.shape[3:])
        h *= 2
    return Y


def sketch_apply_srht(A, seed, iteration, m, problem=0, out_dtype="float64"):
    """S A = (1/sqrt(m)) P H D A for dense A (n x d)."""
    A = np.asarray(A, dtype=np.float64)
    n, d = A.shape
    N = padded_rows(n)
    Y = np.zeros((N, d))
    Y[:n] = srht_signs(seed, iteration, n, problem)[:, None] * A
    Y = fwht(Y)
    rows = srht_rows(seed, iteration, m, N, problem)
    return round_output(Y[rows] * (1.0 / math.sqrt(m)), out_dtype)


def dense_srht_matrix(seed, iteration, n, m, problem=0):
    """Explicit m x n S = (1/sqrt(m)) P H_N[:, :n] D (tiny sizes; brute force)."""
    from scipy.linalg import hadamard
    N = padded_rows(n)
    H = hadamard(N).astype(np.float64)[:, :n]
    rows = srht_rows(seed, iteration, m, N, problem)
    return H[rows] * srht_signs(seed, iteration, n, problem)[None, :] / math.sqrt(m)


# --------------------------------------------------------------------------
# Gaussian
# --------------------------------------------------------------------------
def gaussian_matrix(seed, iteration, m, n, problem=0, with_radius=False):
    """G (m x n) of the Gaussian sketch (before the 1/sqrt(m) scale); with
    with_radius, also the Box-Muller radius rho of every entry (|G| <= rho)."""
    q = (m + 3) // 4
    i = np.arange(n, dtype=np.uint64)
    G = np.empty((4 * q, n))
    R = np.empty((4 * q, n))
    two53 = float(2 ** 53)
    for qq in range(q):
        w = philox4x64(i, qq, problem, STREAM_GAUSSIAN, seed, iteration)
        for h in range(2):
            u1 = ((w[2 * h] >> np.uint64(11)).astype(np.float64) + 1.0) / two53
            u2 = (w[2 * h + 1] >> np.uint64(11)).astype(np.float64) / two53
            rho = np.sqrt(-2.0 * np.log(u1))
            G[4 * qq + 2 * h] = rho * np.cos(2.0 * np.pi * u2)
            G[4 * qq + 2 * h + 1] = rho * np.sin(2.0 * np.pi * u2)
            R[4 * qq + 2 * h] = rho
            R[4 * qq + 2 * h + 1] = rho
    return (G[:m], R[:m]) if with_radius else G[:m]


def sketch_apply_gaussian(A, seed, iteration, m, problem=0, out_dtype="float64"):
    """S A = (1/sqrt(m)) (G A) for dense A (n x d)."""
    A = np.asarray(A, dtype=np.float64)
    G = gaussian_matrix(seed, iteration, m, A.shape[0], problem)
    return round_output((G @ A) * (1.0 / math.sqrt(m)), out_dtype)


def dense_gaussian_matrix(seed, iteration, n, m, problem=0):
    """Explicit m x n S = G / sqrt(m)."""
    return gaussian_matrix(seed, iteration, m, n, problem) / math.sqrt(m)
