"""Input generators (numpy PCG64, seeded).  No recompression arithmetic here.

Workloads (sizes and value laws):

* ``tiny``      d=6, n=4, all ranks 3, cores i.i.d. N(0, 1/(n*r)) with r=3.
* ``spectral``  d=20, n=32, r_x=r_y=20; every core is a Haar-random
                left-orthonormal factor times diag(2^(-j/2)), j=1..r_k.
* ``trig``      d=3, n=256 periodic grid, u = sum of 40 separable products
                of sin/cos with random amplitudes (ranks [1,40,40,1]).
* ``batched``   512 pairs with d in [8,32], n in {16,32,64}, ranks in [8,48],
                cores as in ``spectral``.
* ``power``     Qing and Alpine functions on 10^d grids (d = 10..50) as rank-d
                TTs, for the power iteration that finds their largest entry.
* ``qtt``       QTT (mode size 2, order 3D) trig fields on (2^D)^3 grids, the
                shape of the Allen-Cahn solutions (ranks up to 30).
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
    "power": dict(d=(10, 20, 30, 40, 50), n=10, ell=5, iters=100),
    "qtt": dict(D=(7, 9, 12, 15), terms=15, tol=1e-8),
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


def separable_sum_tt(values: Sequence[np.ndarray]) -> TT:
    """f(x_1..x_d) = sum_k g_k(x_k) on a product grid, from the per-mode
    values g_k (arrays of length n_k), as the rank-d TT of its d separable
    terms (term t is g_t in mode t and 1 elsewhere): ranks [1, d, .., d, 1]."""
    d = len(values)
    cores = []
    for k, g in enumerate(values):
        n = len(g)
        if d == 1:
            cores.append(np.asarray(g, dtype=np.float64).reshape(1, n, 1))
            continue
        lr = 1 if k == 0 else d
        rr = 1 if k == d - 1 else d
        c = np.zeros((lr, n, rr))
        for t in range(d):
            v = g if t == k else np.ones(n)
            if k == 0:
                c[0, :, t] = v
            elif k == d - 1:
                c[t, :, 0] = v
            else:
                c[t, :, t] = v
        cores.append(c)
    return cores


def qing_values(d: int, n: int = 10) -> List[np.ndarray]:
    """Per-mode values of the Qing function sum_i (x_i - i)^2 on n uniform
    points of [-500, 500] (endpoints included), i = 1..d."""
    x = np.linspace(-500.0, 500.0, n)
    return [(x - (i + 1)) ** 2 for i in range(d)]


def alpine_values(d: int, n: int = 10) -> List[np.ndarray]:
    """Per-mode values of the Alpine function sum_i |x_i sin x_i + 0.1 x_i|
    on n uniform points of [-2.5 pi, 2.5 pi] (endpoints included)."""
    x = np.linspace(-2.5 * math.pi, 2.5 * math.pi, n)
    g = np.abs(x * np.sin(x) + 0.1 * x)
    return [g.copy() for _ in range(d)]


def qtt_sine(k: float, D: int) -> TT:
    """sin(k x_j) on the periodic grid x_j = h (j - 1/2), h = 2 pi / 2^D,
    j = 1..2^D, as a QTT of order D (mode sizes 2, ranks 2): with
    j - 1 = sum_b i_b 2^(D-b) (i_1 the most significant bit), the angle is
    k h / 2 + sum_b theta_b i_b, theta_b = k h 2^(D-b), carried as
    [cos, sin] through the rotations of the cores."""
    h = 2.0 * math.pi / (1 << D)
    cores = []
    for b in range(1, D + 1):
        th = k * h * (1 << (D - b))
        c = np.zeros((2, 2, 2))
        for i in (0, 1):
            a = th * i
            c[:, i, :] = [[math.cos(a), math.sin(a)], [-math.sin(a), math.cos(a)]]
        cores.append(c)
    a0 = k * h / 2.0
    first = np.einsum("p,pir->ir", np.array([math.cos(a0), math.sin(a0)]), cores[0])[None, :, :]
    last = np.einsum("pir,r->pi", cores[-1], np.array([0.0, 1.0]))[:, :, None]
    if D == 1:
        return [np.einsum("ir,r->i", first[0], np.array([0.0, 1.0])).reshape(1, 2, 1)]
    return [first] + cores[1:-1] + [last]


def qtt_trig_field(seed: int, D: int, terms: int = 15, kmax: int = 6):
    """phi(x1, x2, x3) = sum_t a_t sin(k_t1 x1) sin(k_t2 x2) sin(k_t3 x3) on
    the (2^D)^3 periodic grid as a QTT of order 3D (mode sizes 2; the D bits
    of x1, then of x2, then of x3), a_t ~ U[0.1, 1.1], k ~ U{1..kmax}; the
    shape of the Allen-Cahn solutions of Sec. 5 (ranks up to 2 terms).
    Returns (cores, amplitudes, frequencies [terms][3])."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.1, 1.1, size=terms)
    ks = rng.integers(1, kmax + 1, size=(terms, 3))
    d = 3 * D
    parts = []
    for t in range(terms):
        cs = []
        for m in range(3):
            cs += qtt_sine(float(ks[t, m]), D)
        cs[0] = cs[0] * a[t]
        parts.append(cs)
    # sum of the terms: first cores side by side, last cores stacked,
    # interior cores block-diagonal
    cores = []
    for k in range(d):
        blocks = [p[k] for p in parts]
        if k == 0:
            cores.append(np.concatenate(blocks, axis=2))
        elif k == d - 1:
            cores.append(np.concatenate(blocks, axis=0))
        else:
            rl = sum(b.shape[0] for b in blocks)
            rr = sum(b.shape[2] for b in blocks)
            c = np.zeros((rl, 2, rr))
            i0 = j0 = 0
            for b in blocks:
                c[i0:i0 + b.shape[0], :, j0:j0 + b.shape[2]] = b
                i0 += b.shape[0]
                j0 += b.shape[2]
            cores.append(c)
    return cores, a, ks


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
