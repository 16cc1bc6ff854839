"""Seeded Gaussian sketch from Philox4x32-10 (oracle side, numpy).

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit
counter and a 2 x 32-bit key; each of 10 rounds multiplies counter words 0
and 2 by the constants 0xD2511F53 and 0xCD9E8D57 (64-bit products split into
high/low halves), mixes them with words 1 and 3 and the key, and the key is
bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.

Sketch definition (the random Gaussian TT of Def. 2.1):
* key = (seed mod 2^32, seed div 2^32);
* element e of core k (row-major over (l_{k-1}, n_k, l_k)) uses counter
  (p mod 2^32, p div 2^32, k, 0x5A7C) with p = e div 2;
* two uniforms in (0,1) with 53 bits each:
  u_a = ((w0 >> 5) 2^26 + (w1 >> 6) + 1/2) 2^-53, u_b likewise from (w2, w3);
* Box-Muller: g0 = sqrt(-2 ln u_a) cos(2 pi u_b) for even e,
  g1 = sqrt(-2 ln u_a) sin(2 pi u_b) for odd e;
* entry = g / sqrt(l_{k-1} n_k l_k)  (variance of Def. 2.1).
"""

from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
STREAM_SKETCH = 0x5A7C


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Inputs are uint32 values or arrays (held in
    uint64 to keep the 64-bit products exact); returns four uint64 arrays
    with values < 2^32."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    sh = np.uint64(32)
    for rnd in range(10):
        p0 = M0 * c0                 # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> sh, p0 & MASK
        hi1, lo1 = p1 >> sh, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
        if rnd < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def gaussian_stream(seed: int, core: int, count: int) -> np.ndarray:
    """The first ``count`` standard normals of core ``core``'s stream."""
    npairs = (count + 1) // 2
    p = np.arange(npairs, dtype=np.uint64)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    w0, w1, w2, w3 = philox4x32_10(p & MASK, p >> np.uint64(32), np.uint64(core),
                                   np.uint64(STREAM_SKETCH), k0, k1)
    two26 = 67108864.0
    inv53 = 1.0 / 9007199254740992.0
    ua = ((w0 >> np.uint64(5)).astype(np.float64) * two26 + (w1 >> np.uint64(6)).astype(np.float64) + 0.5) * inv53
    ub = ((w2 >> np.uint64(5)).astype(np.float64) * two26 + (w3 >> np.uint64(6)).astype(np.float64) + 0.5) * inv53
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * math.pi * ub
    g = np.empty(2 * npairs)
    g[0::2] = rad * np.cos(ang)
    g[1::2] = rad * np.sin(ang)
    return g[:count]


def sketch(seed: int, n: Sequence[int], ell: Sequence[int]) -> List[np.ndarray]:
    """The seeded random Gaussian TT with ranks ``ell`` (Def. 2.1)."""
    d = len(n)
    out = []
    for k in range(d):
        shape = (int(ell[k]), int(n[k]), int(ell[k + 1]))
        cnt = shape[0] * shape[1] * shape[2]
        g = gaussian_stream(seed, k, cnt) / math.sqrt(cnt)
        out.append(g.reshape(shape))
    return out
