"""Philox4x64-10 counter-based generator and the Box-Muller map (oracle side).

Philox4x64-10 follows Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): ten rounds, each multiplying words 0
and 2 by fixed 64-bit constants, xoring the high halves into the other words
with the round key, and bumping the key by two Weyl constants between rounds.
Written here in vectorised numpy on uint64 with an explicit 64x64->128 bit
product; independent of the HIP implementation.

Normal deviates use the Box-Muller transform (Box & Muller, 1958) on the
top 53 bits of words 0 and 1 of one block.
"""
import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """(hi, lo) 64-bit halves of the 128-bit product a*b (uint64 arrays)."""
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply Philox4x64-10 to counters ctr[..., 4] under key (k0, k1)."""
    with np.errstate(over="ignore"):
        c = [np.asarray(ctr[..., w], dtype=np.uint64).copy() for w in range(4)]
        k0 = np.uint64(key[0])
        k1 = np.uint64(key[1])
        for rnd in range(10):
            if rnd:
                k0 = np.uint64((int(k0) + int(_W0)) & 0xFFFFFFFFFFFFFFFF)
                k1 = np.uint64((int(k1) + int(_W1)) & 0xFFFFFFFFFFFFFFFF)
            hi0, lo0 = mulhilo64(_M0, c[0])
            hi1, lo1 = mulhilo64(_M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        return np.stack(c, -1)


def box_muller(x0, x1):
    """Standard normal from two 64-bit words: u1 in (0,1), u2 in [0,1)."""
    two53 = 2.0 ** -53
    u1 = ((x0 >> np.uint64(11)).astype(np.float64) + 0.5) * two53
    u2 = (x1 >> np.uint64(11)).astype(np.float64) * two53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos((2.0 * np.pi) * u2)
