"""Counter-based random numbers for the randomized rounding's sketch cores.

TEST INFRASTRUCTURE ONLY: part of the oracle.  The GPU library draws the same
numbers with its own implementation of the same published generator; the two
share no code.

Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011): a 128-bit counter (four 32-bit words) and a
64-bit key (two words) pass through ten rounds.  Each round multiplies words
0 and 2 of the counter by the round multipliers, keeps both halves of the
64-bit products and mixes them with words 1 and 3 and the key; the key is
bumped by the Weyl constants between rounds.

Sketch entry (the randomized rounding's reading of "a random TT"): entry e of
core `core` in rounding pass `round_index` under key `seed` comes from the
counter (e, core, round_index, 0) and the key (seed mod 2^32, seed div 2^32).
The first two output words give the 53-bit integer x = w0 * 2^21 + (w1 >> 11),
and the entry is x * 2^-52 - 1, uniform on [-1, 1) and exact in FP64.
"""
from __future__ import annotations

import numpy as np

_MUL = (0xD2511F53, 0xCD9E8D57)      # round multipliers
_WEYL = (0x9E3779B9, 0xBB67AE85)     # key increments
_MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """One block of Philox-4x32-10 on Python integers: counter (c0, c1, c2, c3),
    key (k0, k1) -> four 32-bit output words."""
    c = [int(v) & _MASK for v in counter]
    k0, k1 = int(key[0]) & _MASK, int(key[1]) & _MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + _WEYL[0]) & _MASK
            k1 = (k1 + _WEYL[1]) & _MASK
        p0 = _MUL[0] * c[0]
        p1 = _MUL[1] * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c[3] ^ k1) & _MASK, p0 & _MASK]
    return tuple(c)


def _philox_words01(e: np.ndarray, core: int, round_index: int, seed: int):
    """Words 0 and 1 of Philox-4x32-10 for counters (e, core, round_index, 0),
    vectorised over e in uint64 arithmetic (every product of two 32-bit words
    fits)."""
    m = np.uint64(_MASK)
    c0 = e.astype(np.uint64) & m
    c1 = np.full_like(c0, core & _MASK)
    c2 = np.full_like(c0, round_index & _MASK)
    c3 = np.zeros_like(c0)
    k0, k1 = seed & _MASK, (seed >> 32) & _MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + _WEYL[0]) & _MASK
            k1 = (k1 + _WEYL[1]) & _MASK
        p0 = np.uint64(_MUL[0]) * c0
        p1 = np.uint64(_MUL[1]) * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0), p1 & m,
                          (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1), p0 & m)
    return c0, c1


def sketch_entries(seed: int, core: int, round_index: int, n: int) -> np.ndarray:
    """Entries 0 .. n-1 of a sketch core, uniform on [-1, 1)."""
    w0, w1 = _philox_words01(np.arange(n, dtype=np.uint64), core, round_index, seed)
    x = (w0 << np.uint64(21)) | (w1 >> np.uint64(11))
    return x.astype(np.float64) * 2.0 ** -52 - 1.0
