"""Philox4x32-10 and uniform conversions (oracle side).

The paper only requires independent uniform samples in each target element
(sec. 4.1, the uniform-density estimator and algorithm step 3).  The transfer
fixes the generator to make every sample a pure function of
(seed, stream, element, sample index):

* Philox4x32-10 of Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
  as easy as 1, 2, 3" (SC'11): a 4-word counter, a 2-word key, ten rounds of
  two 32x32->64 multiplications, with a Weyl increment of the key between
  rounds.
* 53-bit open-interval doubles: from two words (a, b) take
  m = ((a << 32) | b) >> 12 (52 bits), u = (2m + 1) * 2^-53.  Exact in
  binary64, never 0 or 1.
* 24-bit open-interval floats from the same m: u = (2 (m >> 29) + 1) * 2^-24.

Parity: pinned bit for bit against rocRAND's host Philox4x32-10 generator
(an independent implementation, run as a library) and by the closed-form
range/exactness checks of the conversions.
"""
from __future__ import annotations

import numpy as np

MUL0 = np.uint64(0xD2511F53)
MUL1 = np.uint64(0xCD9E8D57)
WEYL0 = np.uint32(0x9E3779B9)
WEYL1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def _mulhilo(m: np.uint64, x: np.ndarray):
    p = m * x.astype(np.uint64)
    return (p >> np.uint64(32)).astype(np.uint32), (p & MASK32).astype(np.uint32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on counter (c0..c3) with key (k0, k1); all uint32.

    Counters may be arrays (broadcast together); keys are scalars.
    """
    c = [np.asarray(v, dtype=np.uint32) for v in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(MUL0, c[0])
            hi1, lo1 = _mulhilo(MUL1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            k0 = np.uint32(k0 + WEYL0)
            k1 = np.uint32(k1 + WEYL1)
    return c


def key_from_seed(seed: int):
    """Split a 64-bit seed into the two 32-bit key words (low word first)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def mantissa52(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return ((a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)) >> np.uint64(12)


def uniform53(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Open-interval double (2m+1) 2^-53 from words (a, b)."""
    m = mantissa52(a, b)
    return (2 * m + 1).astype(np.float64) * 2.0 ** -53


def uniform24(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Open-interval float (2 (m>>29) + 1) 2^-24 from the same 52-bit m."""
    m = mantissa52(a, b) >> np.uint64(29)
    return ((2 * m + 1).astype(np.float64) * 2.0 ** -24).astype(np.float32)
