"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), written from its published
definition: ten rounds of two 32x32->64 multiplies with the round constants
0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule with 0x9E3779B9 / 0xBB67AE85.

Two backends produce identical bits: numpy (uint64 lanes holding 32-bit values)
and torch (int64 lanes; the 64-bit product may wrap, which leaves the low 64
bits, and therefore both 32-bit halves, intact).  The per-texel visibility
masks of the synthetic scenes are drawn from it so that a mask can be
regenerated on the host for a handful of vertices or on the device for a full
workload and come out the same.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_np(c0, c1, c2, c3, k0, k1, rounds=10):
    """numpy Philox4x32; counters are broadcastable integer arrays < 2**32."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & np.uint64(MASK32)
                      for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(k0 & MASK32)
    k1 = np.uint64(k1 & MASK32)
    m32 = np.uint64(MASK32)
    s32 = np.uint64(32)
    for r in range(rounds):
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> s32, p0 & m32
        hi1, lo1 = p1 >> s32, p1 & m32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        k0 = np.uint64((int(k0) + W0) & MASK32)
        k1 = np.uint64((int(k1) + W1) & MASK32)
    return c0, c1, c2, c3


def philox4x32_torch(c0, c1, c2, c3, k0, k1, rounds=10):
    """torch Philox4x32 on int64 tensors holding values in [0, 2**32)."""
    import torch
    m32 = MASK32
    c0, c1, c2, c3 = torch.broadcast_tensors(c0, c1, c2, c3)
    c0, c1, c2, c3 = (c.to(torch.int64) & m32 for c in (c0, c1, c2, c3))
    k0 = k0 & m32
    k1 = k1 & m32
    for r in range(rounds):
        p0 = c0 * M0          # may wrap modulo 2**64; both halves survive
        p1 = c2 * M1
        hi0, lo0 = (p0 >> 32) & m32, p0 & m32
        hi1, lo1 = (p1 >> 32) & m32, p1 & m32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        k0 = (k0 + W0) & m32
        k1 = (k1 + W1) & m32
    return c0, c1, c2, c3
