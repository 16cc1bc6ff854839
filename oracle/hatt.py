"""HPCRL (Alg. 3) and HaTT (Alg. 4): recompression of y (.) z without the
PKP cores, FP64 numpy.

Index conventions: cores 0-based (c = 0..d-1); bond b = 1..d-1 between
cores b-1 and b; ``W[b]`` is the paper's W^{(b)} (r_b s_b x l_b).  A PKP
row/column index (alpha, beta) is alpha * s + beta (y's index slow, Sec. 2.1).
The paper's fold u|^{s}_{r} is column-major (Sec. 2.1), so for a column u of
length r s, U_gamma[beta, alpha] = u[alpha * s + beta]; ``_fold`` does that.

Reading taken for HaTT-2: the truncated split of W^{(k)} (eq. HPCRL--2) only
feeds the recursion for W^{(k-1)}; the sweep of Alg. 4 multiplies by the
W^{(k)} that was computed (untruncated), so the sketched frame keeps l_k
columns.  The truncation keeps sigma_gamma > ep * ||W^{(k)}||_2 (strict),
and at least one term.
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .tt import _qr_pos

TT = List[np.ndarray]


def _fold(u: np.ndarray, r: int, s: int) -> np.ndarray:
    """u|^{s}_{r}: column-major fold of a length-(r s) vector into s x r."""
    return u.reshape(r, s).T


def _vec(m: np.ndarray) -> np.ndarray:
    """vec(): column-major vectorization (Sec. 2.1)."""
    return m.flatten(order="F")


def wl_column(zi: np.ndarray, u_col: np.ndarray, yi: np.ndarray) -> np.ndarray:
    """One column of W_L (eq. WLWR): vec(Z_k(i) U_gamma Y_k(i)^T)."""
    r, s = yi.shape[1], zi.shape[1]
    return _vec(zi @ _fold(u_col, r, s) @ yi.T)


def core_update_row(zi: np.ndarray, m_row: np.ndarray, yi: np.ndarray) -> np.ndarray:
    """One row of a new core (eq. M*core0):
    X_{k+1}(gamma, i, :) = vec(Z_{k+1}(i)^T M_gamma Y_{k+1}(i))^T."""
    r, s = yi.shape[0], zi.shape[0]
    return _vec(zi.T @ _fold(m_row, r, s) @ yi)


def hpcrl(y: Sequence[np.ndarray], z: Sequence[np.ndarray], rt: Sequence[np.ndarray],
          variant: int = 1, ep: float = 0.0, return_split_ranks: bool = False):
    """Alg. 3.  Returns ``W`` indexed by bond (entry 0 unused); with
    ``return_split_ranks`` also the number of rank-1 terms used per bond."""
    d = len(y)
    w: List[np.ndarray] = [None] * d  # type: ignore[list-item]
    used = [0] * d
    if d < 2:
        return (w, used) if return_split_ranks else w
    # W^{(d-1)} = H(Y_d (x)^1 Z_d) H(R_d)^T; H(Y_d (x)^1 Z_d)(alpha s + beta, i) = Y_d(alpha,i) Z_d(beta,i)
    yd, zd, rd = y[d - 1][:, :, 0], z[d - 1][:, :, 0], rt[d - 1][:, :, 0]
    hyz = (yd[:, None, :] * zd[None, :, :]).reshape(yd.shape[0] * zd.shape[0], -1)
    w[d - 1] = hyz @ rd.T
    for b in range(d - 1, 1, -1):
        c = b - 1
        wb = w[b]
        rk, sk = y[c].shape[2], z[c].shape[2]
        if variant == 1:                       # eq. HPCRL--1: U = W, V = S = I
            u = wb
            vs = np.eye(wb.shape[1])
        elif variant == 2:                     # eq. HPCRL--2: (truncated) SVD
            uu, sg, vt = np.linalg.svd(wb, full_matrices=False)
            keep = int(np.sum(sg > ep * sg[0])) if sg[0] > 0 else 1
            keep = max(1, keep)
            u = uu[:, :keep]
            vs = vt[:keep, :].T * sg[None, :keep]      # sigma_gamma V(:, gamma)
        else:
            raise ValueError("variant must be 1 or 2")
        nterm = u.shape[1]
        used[b] = nterm
        r0, n, _ = y[c].shape
        s0 = z[c].shape[0]
        wl = np.empty((r0 * s0, n * nterm))
        wr = np.empty((rt[c].shape[0], n * nterm))
        ur = u.reshape(rk, sk, nterm)            # ur[alpha, beta, gamma] = U(alpha s + beta, gamma)
        for i in range(n):
            yi, zi, ri = y[c][:, i, :], z[c][:, i, :], rt[c][:, i, :]
            # all gamma at once: vec(Z U_gamma Y^T)[alpha' s0 + beta']
            #   = sum_{alpha, beta} Y(alpha', alpha) Z(beta', beta) U(alpha s + beta, gamma)
            blk = np.einsum("xa,yb,abg->xyg", yi, zi, ur, optimize=True).reshape(r0 * s0, nterm)
            wl[:, i * nterm:(i + 1) * nterm] = blk
            wr[:, i * nterm:(i + 1) * nterm] = ri @ vs          # R_k(i) V(:, gamma)
        w[b - 1] = wl @ wr.T                     # eq. LISRmatrix with S folded into W_R
    return (w, used) if return_split_ranks else w


def hatt(y: Sequence[np.ndarray], z: Sequence[np.ndarray], rt: Sequence[np.ndarray],
         variant: int = 1, ep: float = 0.0) -> TT:
    """Alg. 4 with the sketch TT ``rt`` (ranks l_k) given.  Output ranks are
    the sketch's l_k; cores 1..d-1 are left-orthogonal."""
    d = len(y)
    if [c.shape[1] for c in y] != [c.shape[1] for c in z]:
        raise ValueError("mode sizes differ")
    if d == 1:
        return [(y[0][0, :, 0] * z[0][0, :, 0]).reshape(1, -1, 1)]
    w = hpcrl(y, z, rt, variant, ep)
    # X_1 = Y_1 (x)^3 Z_1: V(X_1)(i, alpha s + beta) = Y_1(i, alpha) Z_1(i, beta)
    y1, z1 = y[0][0], z[0][0]
    xm = (y1[:, :, None] * z1[:, None, :]).reshape(y1.shape[0], -1)
    l_prev = 1
    out: TT = []
    for c in range(d - 1):
        b = c + 1
        n = y[c].shape[1]
        q, _ = _qr_pos(xm @ w[b])                # eq. updatcores1
        lb = q.shape[1]
        out.append(q.reshape(l_prev, n, lb))     # V(X_k) = Q
        m = q.T @ xm                              # M^{(k)} = Q^T X^{(k)}
        rk, sk = y[c].shape[2], z[c].shape[2]
        yn, zn = y[c + 1], z[c + 1]
        r1, n1, r2 = yn.shape
        s1, _, s2 = zn.shape
        mr = m.reshape(lb, rk, sk)               # mr[g, alpha, beta] = M(g, alpha s + beta)
        xn = np.empty((lb, n1, r2 * s2))
        for i in range(n1):
            # row g: vec(Z(i)^T M_g Y(i))[alpha' s2 + beta']
            #   = sum_{alpha, beta} M(g, alpha s + beta) Y(alpha, i, alpha') Z(beta, i, beta')
            xn[:, i, :] = np.einsum("gab,ax,by->gxy", mr, yn[:, i, :], zn[:, i, :], optimize=True).reshape(lb, r2 * s2)
        xm = xn.reshape(lb * n1, r2 * s2)
        l_prev = lb
    out.append(xm.reshape(l_prev, y[d - 1].shape[1], 1))
    return out
