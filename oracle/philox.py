"""Philox4x32-10 counter-based generator (oracle side).

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
Random Numbers: As Easy as 1, 2, 3", SC'11, Sec. 4.2): a 4x32-bit counter and a
2x32-bit key; each of ten rounds multiplies counter words 0 and 2 by fixed
32-bit constants, splits the 64-bit products into high and low halves and
recombines them with the other counter words and the round key; the key is
bumped by the two Weyl constants between rounds.

The paper draws r1, r2 of Eq. (11) as uniform values in [0, 1) without naming a
generator.  This build fixes a counter-based one so that the draws of the GPU
path and of the oracle are the same numbers; the counter layout is stated in
`pso_counter`.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ctr: uint32-compatible array [..., 4]; key: [2] or [..., 2].
    Returns uint32 [..., 4].
    """
    c = np.asarray(ctr, dtype=np.uint64) & MASK
    k = np.broadcast_to(np.asarray(key, dtype=np.uint64) & MASK, c.shape[:-1] + (2,))
    c0, c1, c2, c3 = (c[..., i].copy() for i in range(4))
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    for rnd in range(10):
        p0 = c0 * np.uint64(M0)          # < 2^64: exact in uint64
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if rnd != 9:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed: int):
    """64-bit seed -> Philox key (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & MASK, seed >> 32], dtype=np.uint64)


def u24(w):
    """uint32 word -> uniform double in [0, 1) with 24 bits: (w >> 8) * 2^-24."""
    return (np.asarray(w, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * (2.0 ** -24)


INIT_STREAM = 0xFFFFFFFF   # iteration word used for the initial positions


def pso_counter(tree: int, node: int, t: int, p: int, d: int, D: int):
    """Counter of the draw that serves dimension pair d//2 of particle p.

    Word 0 = p * ceil(D/2) + d//2, word 1 = iteration t (INIT_STREAM for the
    initial positions), word 2 = node id, word 3 = tree id.
    """
    dh = (D + 1) // 2
    return np.array([p * dh + d // 2, t & MASK, node & MASK, tree & MASK], dtype=np.uint64)
