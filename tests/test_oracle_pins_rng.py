"""CPU pins of the oracle's counter-based Gaussian stream (oracle/rng.py):
Philox4x32-10 against its authors' known-answer vectors, the Box-Muller
radius identity, and the distribution of a large sample."""
import math
import os

import numpy as np
import pytest

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = kat_rows()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = rng.philox4x32_10(np.array([ctr], dtype=np.uint32), key)[0]
        assert [int(v) for v in got] == out


def test_philox_is_a_function_of_counter_and_key():
    # one counter word or one key bit changed changes the output (no word is
    # dropped from the rounds)
    base = rng.philox4x32_10(np.array([[1, 2, 3, 4]], dtype=np.uint32), (5, 6))[0]
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert not np.array_equal(rng.philox4x32_10(np.array([c], dtype=np.uint32), (5, 6))[0], base)
    assert not np.array_equal(rng.philox4x32_10(np.array([[1, 2, 3, 4]], dtype=np.uint32), (5, 7))[0], base)
    assert not np.array_equal(rng.philox4x32_10(np.array([[1, 2, 3, 4]], dtype=np.uint32), (4, 6))[0], base)


def test_box_muller_radius_and_layout():
    # samples 4q, 4q+1 share the radius sqrt(-2 ln u1) of word 0; 4q+2, 4q+3
    # that of word 2 (cos^2 + sin^2 = 1)
    seed = 0x123456789
    z = rng.gaussian(seed, 0, 4 * 64)
    q = np.arange(64, dtype=np.uint64)
    ctr = np.zeros((64, 4), dtype=np.uint32)
    ctr[:, 0] = q.astype(np.uint32)
    w = rng.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    for j, word in ((0, 0), (2, 2)):
        u1 = (w[:, word].astype(np.float64) + 0.5) * 2.0 ** -32
        r2 = z[j::4] ** 2 + z[j + 1::4] ** 2
        assert np.allclose(r2, -2.0 * np.log(u1), rtol=1e-13, atol=0)
    # the angle comes from the next word: tan = sin / cos = tan(2 pi u2)
    u2 = (w[:, 1].astype(np.float64) + 0.5) * 2.0 ** -32
    ang = np.arctan2(z[1::4], z[0::4]) % (2 * math.pi)
    assert np.allclose(ang, (2 * math.pi * u2) % (2 * math.pi), atol=1e-12)


def test_offsets_and_high_counter_word():
    seed = 7
    assert np.array_equal(rng.gaussian(seed, 5, 11), rng.gaussian(seed, 0, 16)[5:])
    # a sample index past 2^34 moves the counter's second word
    e = (1 << 34) + 3
    z = rng.gaussian(seed, e, 1)[0]
    w = rng.philox4x32_10(np.array([[0, 1, 0, 0]], dtype=np.uint32), (seed, 0))[0]
    u1 = (float(w[2]) + 0.5) * 2.0 ** -32
    u2 = (float(w[3]) + 0.5) * 2.0 ** -32
    assert z == pytest.approx(math.sqrt(-2 * math.log(u1)) * math.sin(2 * math.pi * u2), rel=1e-14)


def test_gaussian_moments_and_ks():
    from scipy import stats
    z = rng.gaussian(2024, 0, 400000)
    assert abs(z.mean()) < 5 * (1 / math.sqrt(z.size))
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert abs(stats.skew(z)) < 5 * math.sqrt(6 / z.size)
    assert abs(stats.kurtosis(z)) < 5 * math.sqrt(24 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
