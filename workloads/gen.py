"""Input generators (numpy PCG64, seeded).  No recompression arithmetic here.

Workloads (sizes and value laws):

* ``tiny``      d=6, n=4, all ranks 3, cores i.i.d. N(0, 1/(n*r)) with r=3.
* ``spectral``  d=20, n=32, r_x=r_y=20; every core is a Haar-random
                left-orthonormal factor times diag(2^(-j/2)), j=1..r_k.
* ``trig``      d=3, n=256 periodic grid, u = sum of 40 separable products
                of sin/cos with random amplitudes (ranks [1,40,40,1]).
* ``batched``   512 pairs with d in [8,32], n in {16,32,64}, ranks in [8,48],
                cores as in ``spectral``.
"""

from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

TT = List[np.ndarray]

WORKLOADS = {
    "tiny": dict(d=6, n=4, r=3, ell_exact=9, ell_trunc=4),
    "spectral": dict(d=20, n=32, r=20, ell=40, max_rank=30),
    "trig": dict(d=3, n=256, r=40, nfreq=20, tol=1e-8, ell2=96, ell3=128),
    "batched": dict(pairs=512, d=(8, 32), n=(16, 32, 64), r=(8, 48), tol=1e-6),
}


def ranks_of(tt: Sequence[np.ndarray]) -> List[int]:
    return [int(tt[0].shape[0])] + [int(c.shape[2]) for c in tt]


def modes_of(tt: Sequence[np.ndarray]) -> List[int]:
    return [int(c.shape[1]) for c in tt]


def feasible_ranks(n: Sequence[int], r) -> List[int]:
    """Bond ranks [1, r_1, ..., r_{d-1}, 1], each capped by the smaller of
    the products of mode sizes on its two sides (the largest rank a TT of
    these mode sizes can have)."""
    d = len(n)
    rr = [r] * (d + 1) if np.isscalar(r) else list(r)
    out = [1] * (d + 1)
    for k in range(1, d):
        left = math.prod(n[:k])
        right = math.prod(n[k:])
        out[k] = int(min(rr[k], left, right))
    return out


def gaussian_tt(rng: np.random.Generator, n: Sequence[int], ranks: Sequence[int],
                std: float | None = None) -> TT:
    """Cores with i.i.d. N(0, std^2) entries (default std^2 = 1/(n_k r_k))."""
    d = len(n)
    cores = []
    for k in range(d):
        s = std if std is not None else 1.0 / math.sqrt(n[k] * max(ranks[k + 1], ranks[k]))
        cores.append(rng.standard_normal((ranks[k], n[k], ranks[k + 1])) * s)
    return cores


def spectral_tt(rng: np.random.Generator, n: Sequence[int], ranks: Sequence[int]) -> TT:
    """Each core: V(core) = Q diag(2^(-j/2)), Q Haar-distributed with
    orthonormal columns (QR of a Gaussian matrix with diag(R) > 0)."""
    d = len(n)
    cores = []
    for k in range(d):
        m, c = ranks[k] * n[k], ranks[k + 1]
        if m < c:
            raise ValueError(f"core {k}: {m} rows < {c} columns; use feasible_ranks")
        g = rng.standard_normal((m, c))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]
        sig = 2.0 ** (-np.arange(1, c + 1) / 2.0)
        cores.append((q * sig[None, :]).reshape(ranks[k], n[k], c))
    return cores


def gaussian_sketch(rng: np.random.Generator, n: Sequence[int], ell: Sequence[int]) -> TT:
    """Explicit Gaussian TT with ranks ``ell`` and entry variance
    1/(ell_{k-1} n_k ell_k) (the random Gaussian TT of Def. 2.1), drawn with
    numpy so that a caller can pass the same sketch to both sides."""
    d = len(n)
    return [rng.standard_normal((ell[k], n[k], ell[k + 1])) / math.sqrt(ell[k] * n[k] * ell[k + 1])
            for k in range(d)]


def tiny_pair(seed: int, d: int = 6, n: int = 4, r: int = 3):
    """Two TTs of order d, mode size n, all interior ranks r, entries
    N(0, 1/(n r))."""
    rng = np.random.default_rng(seed)
    nn = [n] * d
    rk = feasible_ranks(nn, r)
    std = 1.0 / math.sqrt(n * r)
    return gaussian_tt(rng, nn, rk, std), gaussian_tt(rng, nn, rk, std)


def spectral_pair(seed: int, d: int = 20, n: int | Sequence[int] = 32, rx: int = 20, ry: int = 20):
    rng = np.random.default_rng(seed)
    nn = [n] * d if np.isscalar(n) else list(n)
    return (spectral_tt(rng, nn, feasible_ranks(nn, rx)),
            spectral_tt(rng, nn, feasible_ranks(nn, ry)))


def trig_u(seed: int, n: int = 256, terms: int = 40, nfreq: int = 20) -> TT:
    """u(x1,x2,x3) = sum_t a_t f_{t,1}(x1) f_{t,2}(x2) f_{t,3}(x3) on the
    periodic grid x_j = h (j - 1/2), h = 2 pi / n.  For each mode the
    functions (f_{1,m} .. f_{terms,m}) are a random permutation of
    {cos(jx), sin(jx) : j = 1..nfreq}; a_t ~ U[0.1, 10.1].  The TT has ranks
    [1, terms, terms, 1] (diagonal middle core)."""
    if terms != 2 * nfreq:
        raise ValueError("terms must equal 2*nfreq")
    rng = np.random.default_rng(seed)
    h = 2.0 * math.pi / n
    x = h * (np.arange(n) + 0.5)
    basis = np.empty((2 * nfreq, n))
    for j in range(1, nfreq + 1):
        basis[2 * (j - 1)] = np.cos(j * x)
        basis[2 * (j - 1) + 1] = np.sin(j * x)
    a = rng.uniform(0.1, 10.1, size=terms)
    f = [basis[rng.permutation(2 * nfreq)] for _ in range(3)]  # f[m][t, i]
    c1 = (a[:, None] * f[0]).T[None, :, :]                   # (1, n, T)
    c2 = np.zeros((terms, n, terms))
    for t in range(terms):
        c2[t, :, t] = f[1][t]
    c3 = f[2][:, :, None]                                     # (T, n, 1)
    return [c1, c2, c3]


def batched_pair_shapes(seed: int, pairs: int = 512):
    """Per pair: d ~ U{8..32}, n ~ U{16, 32, 64}, r_x, r_y ~ U{8..48}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(pairs):
        d = int(rng.integers(8, 33))
        n = int(rng.choice([16, 32, 64]))
        out.append((d, n, int(rng.integers(8, 49)), int(rng.integers(8, 49))))
    return out


def mlp_init(seed: int, sizes=((128, 21), (128, 128), (2, 128))) -> np.ndarray:
    """Initial parameters of the width predictor, packed as W1 b1 W2 b2 W3
    b3 (row-major): weights uniform in +-sqrt(6 / (fan_in + fan_out))
    (Glorot and Bengio, 2010), biases zero.  FP64; callers cast."""
    rng = np.random.default_rng(seed)
    parts = []
    for fo, fi in sizes:
        a = np.sqrt(6.0 / (fi + fo))
        parts.append(rng.uniform(-a, a, size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts)
