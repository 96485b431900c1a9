"""Oracle of the on-device image degradation (Alg. 1, step 3, degradImage).

TEST INFRASTRUCTURE ONLY (see the package docstring). The paper names degradImage
without defining it; the reading used throughout: additive Gaussian noise of standard
deviation sigma (grey levels), rounded half-to-even and clipped to [0, M], then salt and
pepper: each pixel independently with probability `density` becomes 0 or M (one half
each).

Random numbers: the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011), written here from its published
definition. Pixel p of stream s draws one block: counter (p mod 2^32, p div 2^32, s, 0),
key (seed mod 2^32, seed div 2^32), output words r0..r3.
  u1 = (r0 + 1) / 2^32 in (0, 1], u2 = r1 / 2^32 in [0, 1)
  z  = sqrt(-2 ln u1) cos(2 pi u2)                       (Box-Muller, float64)
  g  = clip(rint(x + sigma z), 0, M)
  impulse when r2 < floor(density 2^32); then g = M if r3 is odd else 0.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds. ctr: (N, 4) uint32 counters; key: two uint32 words.
    Each round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products), new counter
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key advances by the Weyl constants
    between rounds."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4) & MASK32
    c0, c1, c2, c3 = c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy()
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def pixel_blocks(h: int, w: int, seed: int, stream: int) -> np.ndarray:
    """(h * w, 4) Philox output words of every pixel (row-major pixel index)."""
    p = np.arange(h * w, dtype=np.uint64)
    ctr = np.stack([p & MASK32, p >> np.uint64(32), np.full_like(p, stream & 0xFFFFFFFF),
                    np.zeros_like(p)], axis=1)
    return philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))


def degrade(clean: np.ndarray, sigma: float, density: float, max_value: int, seed: int,
            stream: int = 0, return_pre: bool = False):
    """Noisy integer image (int32) from a clean integer image; with return_pre also the
    unrounded Gaussian stage x + sigma z (float64), for tie checks."""
    x = np.asarray(clean, dtype=np.float64)
    h, w = x.shape
    r = pixel_blocks(h, w, seed, stream).astype(np.float64)
    u1 = (r[:, 0] + 1.0) / 4294967296.0
    u2 = r[:, 1] / 4294967296.0
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    pre = x.reshape(-1) + sigma * z
    g = np.clip(np.rint(pre), 0, max_value)
    thr = np.floor(density * 4294967296.0)
    imp = r[:, 2] < thr
    g = np.where(imp, np.where(r[:, 3].astype(np.uint64) & np.uint64(1), max_value, 0), g)
    g = g.reshape(h, w).astype(np.int32)
    return (g, pre.reshape(h, w)) if return_pre else g
