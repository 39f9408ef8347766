"""Philox4x64-10, written from its published definition (Salmon, Moraes, Dror
and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes no random number generator; the s-hashing matrix and the sign
diagonal only have to be drawn independently and uniformly.  This library draws
them from Philox4x64-10 so that the GPU and this oracle can produce the same
bits independently.  The block function maps a 256-bit counter and a 128-bit
key to 256 output bits through ten rounds of

    (c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))

with the key bumped by the Weyl constants (W0, W1) between rounds.

Pinned in the tests against numpy.random.Philox, an independent library
implementation of the same generator (numpy advances its counter by one before
producing a block, so its first block for counter c is ours for c + 1).
"""

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 128-bit product of two uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    p0 = a_lo * b_lo
    p1 = a_lo * b_hi
    p2 = a_hi * b_lo
    p3 = a_hi * b_hi
    mid = (p0 >> _S32) + (p1 & _LO32) + (p2 & _LO32)
    hi = p3 + (p1 >> _S32) + (p2 >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (p0 & _LO32)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Vectorised block function: counters (c0..c3) and key (k0, k1), all
    broadcastable uint64 arrays.  Returns the four 64-bit output words."""
    with np.errstate(over="ignore"):
        c0 = np.asarray(c0, dtype=np.uint64)
        c1 = np.asarray(c1, dtype=np.uint64)
        c2 = np.asarray(c2, dtype=np.uint64)
        c3 = np.asarray(c3, dtype=np.uint64)
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo64(M0, c0)
            hi1, lo1 = mulhilo64(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3
