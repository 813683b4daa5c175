"""Counter-based Gaussian test-matrix entries, FP64 (oracle).

Test infrastructure: see oracle/__init__.py.

Algorithm RandNysAppx starts from a standard Gaussian test matrix.  When the
library draws it on the device, this module is the independent CPU statement
of the same stream, written from the published definitions:

  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
    easy as 1, 2, 3", SC 2011): a 128-bit counter (four 32-bit words) and a
    64-bit key (two words) go through ten rounds; a round multiplies words 0
    and 2 by the constants 0xD2511F53 and 0xCD9E8D57 (full 64-bit products
    split into high and low halves) and returns (hi_b ^ x1 ^ k0, lo_b,
    hi_a ^ x3 ^ k1, lo_a), where (hi_a, lo_a) is the product of word 0 and
    (hi_b, lo_b) that of word 2; between rounds the key words grow by the
    Weyl constants 0x9E3779B9 and 0xBB67AE85 (mod 2^32).
  * Box-Muller (Box and Muller, 1958): two uniforms u1, u2 in (0, 1) give
    sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2).

Stream layout (the library's convention): sample e of seed s comes from the
Philox call with counter (q mod 2^32, q div 2^32, 0, 0), q = e div 4, and key
(s mod 2^32, s div 2^32); with its output words (w0, w1, w2, w3), samples 4q
and 4q + 1 are the Box-Muller pair of u1 = (w0 + 1/2) 2^-32 and
u2 = (w1 + 1/2) 2^-32, samples 4q + 2 and 4q + 3 that of w2 and w3.

Pins (tests/test_oracle_pins_rng.py): the Philox known-answer vectors that
the generator's authors publish with their library, the radius identity of
Box-Muller (z_even^2 + z_odd^2 = -2 ln u1), and the first four moments and a
two-sided Kolmogorov-Smirnov test of a large sample against N(0, 1).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """ctr: (N, 4) uint32 counters, key: two 32-bit words -> (N, 4) uint32."""
    x = np.asarray(ctr, dtype=np.uint32).astype(np.uint64)
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    x0, x1, x2, x3 = x[:, 0], x[:, 1], x[:, 2], x[:, 3]
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        pa = _M0 * x0
        pb = _M1 * x2
        hi_a, lo_a = pa >> np.uint64(32), pa & _MASK
        hi_b, lo_b = pb >> np.uint64(32), pb & _MASK
        x0, x1, x2, x3 = (hi_b ^ x1 ^ np.uint64(k0), lo_b, hi_a ^ x3 ^ np.uint64(k1), lo_a)
    return np.stack([x0, x1, x2, x3], axis=1).astype(np.uint32)


def box_muller(w_a: np.ndarray, w_b: np.ndarray):
    """Two uint32 words -> the Box-Muller pair (cos branch, sin branch)."""
    u1 = (w_a.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (w_b.astype(np.float64) + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2)


def gaussian(seed: int, offset: int, count: int) -> np.ndarray:
    """Samples offset .. offset + count - 1 of the stream of `seed` (FP64)."""
    if count <= 0:
        return np.zeros(0)
    e = np.arange(offset, offset + count, dtype=np.uint64)
    q = np.unique(e // np.uint64(4))
    ctr = np.zeros((q.size, 4), dtype=np.uint32)
    ctr[:, 0] = (q & _MASK).astype(np.uint32)
    ctr[:, 1] = (q >> np.uint64(32)).astype(np.uint32)
    words = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    z = np.empty((q.size, 4))
    z[:, 0], z[:, 1] = box_muller(words[:, 0], words[:, 1])
    z[:, 2], z[:, 3] = box_muller(words[:, 2], words[:, 3])
    flat = z.reshape(-1)
    start = int(offset - int(q[0]) * 4)
    return flat[start:start + count].copy()
