"""Pins for the oracle's hash: numpy's own Philox4x64-10 stream, exact 128-bit
products, and the distribution the sparse embeddings of Sec. 2 require
(uniform sketch row, equiprobable sign, independent blocks)."""
import numpy as np
import pytest
from scipy import stats

from oracle.philox import mulhilo64, philox4x64, philox4x64_scalar
from oracle.sketch import sketch_hash

MASK = (1 << 64) - 1


def numpy_block(counter, key):
    """numpy's Philox increments its counter before each block, so the block
    of counter c comes from a generator started at c - 1 (256-bit borrow)."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & MASK for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return tuple(int(v) for v in bg.random_raw(4))


CASES = [
    ((1, 0, 0, 0), (1, 2)),
    ((0, 0, 0, 0), (0, 0)),
    ((12345, 3, 7, 0), (20192031, 17)),
    ((MASK, MASK, MASK, MASK), (MASK, MASK)),
    ((0, 1, 0, 0), (99, 0)),
    ((2 ** 40 + 5, 0, 63, 0), (2 ** 63 + 11, 2 ** 32)),
]


@pytest.mark.parametrize("counter,key", CASES)
def test_philox_scalar_matches_numpy(counter, key):
    assert philox4x64_scalar(counter, key) == numpy_block(counter, key)


def test_philox_vector_matches_scalar():
    g = np.random.default_rng(5)
    c0 = g.integers(0, 2 ** 63, size=64, dtype=np.uint64)
    c1 = g.integers(0, 4, size=64, dtype=np.uint64)
    key = (987654321987, 42)
    w = philox4x64(c0, c1, 3, 0, *key)
    for i in range(64):
        ref = philox4x64_scalar((int(c0[i]), int(c1[i]), 3, 0), key)
        assert tuple(int(x[i]) for x in w) == ref


def test_mulhilo64_exact():
    g = np.random.default_rng(6)
    a = g.integers(0, 2 ** 64, size=2000, dtype=np.uint64, endpoint=False)
    b = g.integers(0, 2 ** 64, size=2000, dtype=np.uint64, endpoint=False)
    a[:3] = [MASK, MASK, 0]
    b[:3] = [MASK, 1, MASK]
    hi, lo = mulhilo64(a, b)
    for i in range(len(a)):
        p = int(a[i]) * int(b[i])
        assert int(hi[i]) == p >> 64 and int(lo[i]) == p & MASK


def test_bucket_is_multiply_shift_of_first_word():
    n, m, seed, it = 50, 777, 31, 4
    bucket, sign = sketch_hash(seed, it, n, m, 1)
    for i in range(n):
        w = philox4x64_scalar((i, 0, 0, 0), (seed, it))
        assert bucket[i, 0] == (w[0] * m) >> 64
        assert sign[i, 0] == (-1 if w[1] >> 63 else 1)


def test_sjlt_blocks_use_word_pairs_and_offsets():
    n, m, s, seed, it = 40, 64, 4, 8, 2
    bucket, sign = sketch_hash(seed, it, n, m, s)
    mb = m // s
    for i in range(n):
        for k in range(s):
            w = philox4x64_scalar((i, k // 2, 0, 0), (seed, it))
            wb, ws = w[2 * (k % 2)], w[2 * (k % 2) + 1]
            assert bucket[i, k] == k * mb + ((wb * mb) >> 64)
            assert sign[i, k] == (-1 if ws >> 63 else 1)


def test_bucket_uniform_and_sign_balanced():
    n, m = 1_000_000, 1000
    bucket, sign = sketch_hash(7, 0, n, m, 1)
    counts = np.bincount(bucket[:, 0], minlength=m)
    chi2 = ((counts - n / m) ** 2 / (n / m)).sum()
    assert stats.chi2.sf(chi2, m - 1) > 1e-4
    z = sign.sum() / np.sqrt(n)
    assert abs(z) < 4.5


def test_sjlt_blocks_independent():
    n, m, s = 400_000, 64, 4
    bucket, sign = sketch_hash(11, 3, n, m, s)
    mb = m // s
    for k in range(s):
        assert bucket[:, k].min() >= k * mb and bucket[:, k].max() < (k + 1) * mb
    # joint distribution of the local rows of blocks 0 and 1 is uniform on mb^2
    joint = (bucket[:, 0] - 0) * mb + (bucket[:, 1] - mb)
    counts = np.bincount(joint, minlength=mb * mb)
    chi2 = ((counts - n / mb ** 2) ** 2 / (n / mb ** 2)).sum()
    assert stats.chi2.sf(chi2, mb * mb - 1) > 1e-4
    # signs of blocks 2 and 3 uncorrelated
    assert abs((sign[:, 2].astype(float) * sign[:, 3]).sum() / np.sqrt(n)) < 4.5


def test_keys_and_problems_give_distinct_streams():
    a, _ = sketch_hash(1, 0, 1000, 1 << 20, 1)
    b, _ = sketch_hash(1, 1, 1000, 1 << 20, 1)
    c, _ = sketch_hash(2, 0, 1000, 1 << 20, 1)
    d, _ = sketch_hash(1, 0, 1000, 1 << 20, 1, problem=1)
    for other in (b, c, d):
        assert (a != other).mean() > 0.99


def test_sjlt_requires_divisible_m():
    with pytest.raises(ValueError):
        sketch_hash(0, 0, 10, 10, 4)
