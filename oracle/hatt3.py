"""HaTT for three factors: recompression of x (.) y (.) w without the
three-way PKP cores, FP64 numpy.  Test infrastructure, like all of oracle/.

The paper states the two-factor method (Alg. 3 HPCRL, Alg. 4 HaTT) through
the identity (A kron B) vec(U) = vec(B U A^T) of eq. (kronecker_product_times_vec).
With three factors the Hadamard product's cores are the three-way partial
Kronecker products (rank r_k s_k t_k) and the same identity, applied mode by
mode, gives
  (X kron Y kron W) u = the three-mode product of the r' x s' x t' tensor
                        folded from u with X, Y and W,
so HPCRL's recursion and the sweep's core update become three-mode products
instead of two-sided ones.  Nothing else changes: this is RandOrth (Alg. 2)
on the three-way PKP train with the sketch applied right to left, computed
without forming those cores.  The paper applies its products one pair at a
time (the Allen-Cahn nonlinearity of Sec. 5, Example 4, as successive
products); the three-factor form is an extension, pinned against RandOrth on
the explicit three-way PKP cores.

Index convention: a three-way PKP row/column index (alpha, beta, delta) is
(alpha s + beta) t + delta, the first factor's index slowest (as the two-factor
convention, applied twice).  Cores are 0-based; ``W[b]`` is the sketch matrix
of bond b (r_b s_b t_b x l_b).
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .tt import _qr_pos, modes

TT = List[np.ndarray]


def pkp3_core(x: np.ndarray, y: np.ndarray, w: np.ndarray) -> np.ndarray:
    """A((a s + b) t + c, i, (a' s' + b') t' + c') = X(a,i,a') Y(b,i,b') W(c,i,c'):
    slice i is kron(kron(X(:, i, :), Y(:, i, :)), W(:, i, :))."""
    r0, n, r1 = x.shape
    s0, _, s1 = y.shape
    t0, _, t1 = w.shape
    out = np.empty((r0 * s0 * t0, n, r1 * s1 * t1))
    for i in range(n):
        out[:, i, :] = np.kron(np.kron(x[:, i, :], y[:, i, :]), w[:, i, :])
    return out


def pkp3(x: Sequence[np.ndarray], y: Sequence[np.ndarray], w: Sequence[np.ndarray]) -> TT:
    """TT cores of x (.) y (.) w, ranks r_k s_k t_k."""
    if modes(x) != modes(y) or modes(x) != modes(w):
        raise ValueError("mode sizes differ")
    return [pkp3_core(a, b, c) for a, b, c in zip(x, y, w)]


def hpcrl3(x: Sequence[np.ndarray], y: Sequence[np.ndarray], w: Sequence[np.ndarray],
           rt: Sequence[np.ndarray]) -> List[np.ndarray]:
    """HPCRL (Alg. 3, the HaTT-1 split U = W) for three factors: the sketch
    matrices W^{(k)} of the three-way product, right to left.  Returns a list
    indexed by bond (entry 0 unused)."""
    d = len(x)
    out: List[np.ndarray] = [None] * d  # type: ignore[list-item]
    if d < 2:
        return out
    # last core: rows (a, b, c) of the right-rank-1 cores, one column per i
    xd, yd, wd = x[d - 1][:, :, 0], y[d - 1][:, :, 0], w[d - 1][:, :, 0]
    h = (xd[:, None, None, :] * yd[None, :, None, :] * wd[None, None, :, :]).reshape(-1, xd.shape[1])
    out[d - 1] = h @ rt[d - 1][:, :, 0].T
    for b in range(d - 1, 1, -1):
        c = b - 1
        r1, s1, t1 = x[c].shape[2], y[c].shape[2], w[c].shape[2]
        r0, n, _ = x[c].shape
        s0, t0 = y[c].shape[0], w[c].shape[0]
        u = out[b].reshape(r1, s1, t1, -1)            # u[a', b', c', g] = W^{(k)}((a' s1 + b') t1 + c', g)
        acc = np.zeros((r0 * s0 * t0, rt[c].shape[0]))
        for i in range(n):
            # (X(i) kron Y(i) kron W(i)) applied to every column of W^{(k)}
            blk = np.einsum("xa,yb,zc,abcg->xyzg", x[c][:, i, :], y[c][:, i, :], w[c][:, i, :], u,
                            optimize=True).reshape(r0 * s0 * t0, -1)
            acc += blk @ rt[c][:, i, :].T                # times R_k(i)^T, summed over i
        out[b - 1] = acc
    return out


def hatt3(x: Sequence[np.ndarray], y: Sequence[np.ndarray], w: Sequence[np.ndarray],
          rt: Sequence[np.ndarray]) -> TT:
    """Alg. 4 for three factors with the sketch TT ``rt`` (ranks l_k) given.
    Output ranks are the sketch's l_k; cores 1..d-1 are left-orthogonal."""
    d = len(x)
    if modes(x) != modes(y) or modes(x) != modes(w):
        raise ValueError("mode sizes differ")
    if d == 1:
        return [(x[0][0, :, 0] * y[0][0, :, 0] * w[0][0, :, 0]).reshape(1, -1, 1)]
    wk = hpcrl3(x, y, w, rt)
    x1, y1, w1 = x[0][0], y[0][0], w[0][0]
    # first frame: row i, column (a, b, c) = X_1(i, a) Y_1(i, b) W_1(i, c)
    xm = (x1[:, :, None, None] * y1[:, None, :, None] * w1[:, None, None, :]).reshape(x1.shape[0], -1)
    l_prev = 1
    out: TT = []
    for c in range(d - 1):
        n = x[c].shape[1]
        q, _ = _qr_pos(xm @ wk[c + 1])               # sketched frame, economy QR
        lb = q.shape[1]
        out.append(q.reshape(l_prev, n, lb))
        m = q.T @ xm                                  # M = Q^T X^{(k)}
        r1, s1, t1 = x[c].shape[2], y[c].shape[2], w[c].shape[2]
        xn_, yn_, wn_ = x[c + 1], y[c + 1], w[c + 1]
        n1 = xn_.shape[1]
        r2, s2, t2 = xn_.shape[2], yn_.shape[2], wn_.shape[2]
        mr = m.reshape(lb, r1, s1, t1)
        xn = np.empty((lb, n1, r2 * s2 * t2))
        for i in range(n1):
            # row g of slice i: the three-mode product of M_g with X(i)^T, Y(i)^T, W(i)^T
            xn[:, i, :] = np.einsum("gabc,ax,by,cz->gxyz", mr, xn_[:, i, :], yn_[:, i, :], wn_[:, i, :],
                                    optimize=True).reshape(lb, -1)
        xm = xn.reshape(lb * n1, -1)
        l_prev = lb
    out.append(xm.reshape(l_prev, x[d - 1].shape[1], 1))
    return out
