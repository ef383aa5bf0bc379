"""Philox4x32-10 in vectorised numpy -- a second, independent oracle-side implementation.

TEST INFRASTRUCTURE: used only by the tests to cross-check the C oracle's generator.

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): four 32-bit words and a two-word key; each of the
10 rounds forms the 64-bit products M0*w0 and M1*w2 and maps
(w0, w1, w2, w3) -> (hi(M1 w2) ^ w1 ^ k0, lo(M1 w2), hi(M0 w0) ^ w3 ^ k1, lo(M0 w0));
the key advances by the Weyl constants (W0, W1) between rounds.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
SHIFT32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: uint32 array [..., 4]; key: uint32 array [..., 2] (broadcastable).
    Returns uint32 array [..., 4]."""
    ctr = np.asarray(ctr, dtype=np.uint32)
    key = np.asarray(key, dtype=np.uint32)
    w = [ctr[..., j].astype(np.uint64) for j in range(4)]
    k0 = key[..., 0].astype(np.uint32)
    k1 = key[..., 1].astype(np.uint32)
    for rnd in range(10):
        p0 = M0 * w[0]
        p1 = M1 * w[2]
        hi0, lo0 = p0 >> SHIFT32, p0 & MASK32
        hi1, lo1 = p1 >> SHIFT32, p1 & MASK32
        w = [hi1 ^ w[1] ^ k0.astype(np.uint64), lo1, hi0 ^ w[3] ^ k1.astype(np.uint64), lo0]
        if rnd < 9:
            with np.errstate(over="ignore"):
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
    return np.stack([x.astype(np.uint32) for x in np.broadcast_arrays(*w)], axis=-1)
