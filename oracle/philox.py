"""Philox4x64-10, written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11: a 4x64-bit counter, a 2x64-bit key, ten rounds of the Philox S-box
    (hi0, lo0) = mulhilo(M0, x0);  (hi1, lo1) = mulhilo(M1, x2)
    x <- (hi1 ^ x1 ^ k0,  lo1,  hi0 ^ x3 ^ k1,  lo0)
with the key advanced by the Weyl constants between rounds.

The paper draws Omega from "a random number generator" (Sec. III, Alg. 3
step 1); this counter-based generator is the reading used on both sides so
that host and device draw the same Omega (see ``normal``).

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo).

    Schoolbook multiplication on 32-bit halves; every partial product fits in
    64 bits, carries are propagated explicitly.
    """
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _MASK32, a >> _S32
    b_lo, b_hi = b & _MASK32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _MASK32) + (hl & _MASK32)
    lo = (ll & _MASK32) | ((mid & _MASK32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply the 10-round Philox4x64 bijection.

    ctr: uint64 array of shape (..., 4); key: uint64 pair (k0, k1) or array of
    shape (..., 2). Returns a uint64 array of shape (..., 4).
    """
    with np.errstate(over="ignore"):
        ctr = np.asarray(ctr, dtype=np.uint64)
        key = np.asarray(key, dtype=np.uint64)
        x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
        k0 = np.broadcast_to(key[..., 0], x0.shape).copy()
        k1 = np.broadcast_to(key[..., 1], x0.shape).copy()
        for r in range(10):
            hi0, lo0 = mulhilo64(M0, x0)
            hi1, lo1 = mulhilo64(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            if r != 9:
                k0 = k0 + W0
                k1 = k1 + W1
        return np.stack([x0, x1, x2, x3], axis=-1)


def block_words(seed, stream, blocks, word2=0):
    """Philox output for counters (b, 0, word2, 0), b in ``blocks``, key (seed, stream)."""
    blocks = np.asarray(blocks, dtype=np.uint64)
    ctr = np.zeros(blocks.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = blocks
    ctr[..., 2] = np.uint64(word2)
    return philox4x64_10(ctr, np.array([seed, stream], dtype=np.uint64))
