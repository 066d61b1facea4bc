"""Oracle: Philox4x32-10 counter-based generator and Box-Muller normals (test infrastructure).

Definition from Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11): a round maps counter (c0, c1, c2, c3) with key
(k0, k1) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by (0x9E3779B9,
0xBB67AE85) between rounds; ten rounds.

Start states are i.i.d. N(0,1) (the paper says only "randomly generated",
Sec. III; this is the reading).  Element (s, j) of a [D][b] block with seed
uses counter (s, j, 0, 0) and key (seed_lo, seed_hi); u1 and u2 are the top
53 bits of (r0:r1) and (r2:r3) offset by half an ulp, and
z = sqrt(-2 ln u1) cos(2 pi u2).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 arrays; returns four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def gaussian_block(D, b, seed):
    """[D][b] block of N(0,1) values from Philox4x32-10 + Box-Muller (FP64)."""
    s = np.repeat(np.arange(D, dtype=np.uint64), b)
    j = np.tile(np.arange(b, dtype=np.uint64), D)
    seed = int(seed)
    r0, r1, r2, r3 = philox4x32_10(s, j, 0, 0, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    a = (r0.astype(np.uint64) << np.uint64(32)) | r1.astype(np.uint64)
    c = (r2.astype(np.uint64) << np.uint64(32)) | r3.astype(np.uint64)
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = ((c >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return z.reshape(D, b)
