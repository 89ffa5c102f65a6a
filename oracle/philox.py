"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
published definition.

The paper leaves the hash family of CountSketch and SJLT open (Sec. 2 asks only
for a uniform row h(i) and an equiprobable sign per column of S). This library
fixes Philox4x64-10 so a sketch is a pure function of (seed, iteration, row).

One round maps counter (x0, x1, x2, x3) under key (k0, k1) to
    (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))
and the key is advanced by the Weyl constants between rounds.

Two implementations: `philox4x64_scalar` uses Python integers (the reference
for a handful of counters) and `philox4x64` is the same map vectorised over
numpy uint64 arrays, with the 128-bit product split into 32-bit halves.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
ROUNDS = 10
MASK64 = (1 << 64) - 1


def philox4x64_scalar(counter, key, rounds=ROUNDS):
    """Philox4x64 on Python ints. counter: 4 ints, key: 2 ints (all < 2^64)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return (x0, x1, x2, x3)


_U32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _U32, a >> _S32
    b_lo, b_hi = b & _U32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _U32) + (hl & _U32)
    lo = (ll & _U32) | ((mid & _U32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox4x64: counter words and key words broadcast together.
    Returns four uint64 arrays."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
        x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        m0, m1 = np.uint64(M0), np.uint64(M1)
        w0, w1 = np.uint64(W0), np.uint64(W1)
        for r in range(rounds):
            if r:
                k0 = k0 + w0
                k1 = k1 + w1
            hi0, lo0 = mulhilo64(m0, x0)
            hi1, lo1 = mulhilo64(m1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3
