"""Philox4x32-10 counter-based generator and Box-Muller normals (numpy, uint64 math).

Test infrastructure (see ``oracle/__init__``).

Written from the published definition: Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11 (2011).  A round maps counter
(c0, c1, c2, c3) with key (k0, k1) to
  (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by the Weyl constants
(0x9E3779B9, 0xBB67AE85) between rounds; 10 rounds.

White-noise layout used by the method's seeded initial conditions (a reading: the
paper takes its initial seed from 2LPTic): value p of the grid comes from block
g = p // 4 with counter (g mod 2^32, g // 2^32, 0, 0) and key (seed mod 2^32,
seed // 2^32).  The block's outputs (r0, r1, r2, r3) give two Box-Muller pairs:
u1 = ((r >> 8) + 1) 2^-24 in (0, 1], u2 = (r' >> 8) 2^-24 in [0, 1),
z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) for (r, r') = (r0, r1) -> values
4g, 4g+1 and (r2, r3) -> values 4g+2, 4g+3.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (4, n) uint32-valued array, key: (2, n) or (2,) -> (4, n) uint32."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c])


def white_noise_bits(seed: int, count: int) -> np.ndarray:
    """The raw Philox outputs for values 0..count-1 (count rounded up to 4)."""
    nblk = (count + 3) // 4
    g = np.arange(nblk, dtype=np.uint64)
    ctr = (g & MASK, g >> np.uint64(32), np.zeros_like(g), np.zeros_like(g))
    key = (np.uint64(seed) & MASK, np.uint64(seed) >> np.uint64(32))
    return philox4x32_10(ctr, key)


def white_noise(seed: int, count: int) -> np.ndarray:
    """count N(0, 1) values (FP64) in the layout described in the module docstring."""
    r = white_noise_bits(seed, count).astype(np.float64)
    out = np.empty((r.shape[1], 4))
    for j, (ra, rb) in enumerate(((0, 1), (2, 3))):
        u1 = (np.floor(r[ra] / 256.0) + 1.0) * 2.0**-24
        u2 = np.floor(r[rb] / 256.0) * 2.0**-24
        rad = np.sqrt(-2.0 * np.log(u1))
        out[:, 2 * j] = rad * np.cos(2.0 * np.pi * u2)
        out[:, 2 * j + 1] = rad * np.sin(2.0 * np.pi * u2)
    return out.reshape(-1)[:count]
