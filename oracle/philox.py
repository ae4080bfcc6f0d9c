"""Philox4x32-10 in plain integer arithmetic (oracle; test infrastructure only).

Written from the published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter
and a 2 x 32-bit key; each of the 10 rounds multiplies counter words 0 and 2
by the round constants, swaps and xors the high halves with the other two
words and the key; the key is bumped by the Weyl constants between rounds.
NumPy uint64 holds every 32 x 32 -> 64-bit product exactly.
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """counter: uint [..., 4]; key: uint [..., 2] (broadcast).  Returns the
    four uint32 output words [..., 4]."""
    c = np.asarray(counter, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0 = np.broadcast_to(k[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], c0.shape).copy()
    m0, m1 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK
        p0 = m0 * c0
        p1 = m1 * c2
        c0, c1, c2, c3 = ((p1 >> s32) ^ c1 ^ k0, p1 & _MASK, (p0 >> s32) ^ c3 ^ k1, p0 & _MASK)
    return np.stack([c0, c1, c2, c3], -1).astype(np.uint32)
