"""TT-Rounding, Alg. 1 (Sec. 2.3), FP64 numpy; its truncation loop run from
the right on a left-orthogonal train (tt_round_left_orth, used after Alg. 4
and Alg. 2, whose outputs are left-orthogonal).

Readings (the printed listing is garbled in two places; the meaning taken):

* After the right-to-left loop the listing re-sets the first core to the
  input's first core; that would drop the R factor absorbed at k = 2, so it is
  read as a no-op (core 1 keeps the absorbed factor).
* The left-to-right update multiplies the *orthogonalized* next core (the
  working core B_{k+1}), not the input's core A_{k+1}.
* Truncation rule per bond k (the paper fixes target ranks; a tolerance is
  added the way TT-SVD does it): delta = tol * ||A||_F / sqrt(d-1);
  rho_tol = smallest rho >= 1 with sum_{j > rho} sigma_j^2 <= delta^2
  (tol <= 0 keeps every singular value); rho = min(rho_tol, max_rank[k]).
"""

from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np

from .tt import H, V, _qr_pos, orthogonalize_rl

TT = List[np.ndarray]


def choose_rank(sigma: np.ndarray, delta: float, cap: Optional[int]) -> int:
    """Rank kept at one bond: the smallest rho whose discarded tail
    sum_{j>rho} sigma_j^2 is <= delta^2 (tail summed from the smallest
    singular value up), then capped."""
    m = len(sigma)
    rho = m
    if delta > 0:
        tail = 0.0
        rho = m
        for j in range(m - 1, 0, -1):          # try dropping sigma_j (0-based)
            tail += sigma[j] ** 2
            if tail <= delta * delta:
                rho = j
            else:
                break
    if cap is not None:
        rho = min(rho, int(cap))
    return max(1, rho)


def tt_round(tt: Sequence[np.ndarray], max_rank=None, tol: float = 0.0, return_sigmas: bool = False):
    """Alg. 1.  ``max_rank`` is None, an int (all bonds) or a list of d+1
    bond caps (entries 0 and d ignored).  Returns the rounded TT (and, if
    asked, the singular values seen at each bond)."""
    d = len(tt)
    if max_rank is None:
        caps = [None] * (d + 1)
    elif np.isscalar(max_rank):
        caps = [int(max_rank)] * (d + 1)
    else:
        caps = list(max_rank)
    b = orthogonalize_rl(tt)                      # right-to-left loop of Alg. 1
    nrm = float(np.linalg.norm(b[0]))
    delta = tol * nrm / math.sqrt(d - 1) if (tol > 0 and d > 1) else 0.0
    sigmas = []
    for k in range(d - 1):                        # left-to-right loop
        r0, n, r1 = b[k].shape
        q, r = _qr_pos(V(b[k]))
        u, s, vt = np.linalg.svd(r, full_matrices=False)
        rho = choose_rank(s, delta, caps[k + 1])
        sigmas.append(s)
        b[k] = (q @ u[:, :rho]).reshape(r0, n, rho)
        _, pn, p1 = b[k + 1].shape
        b[k + 1] = ((s[:rho, None] * vt[:rho, :]) @ H(b[k + 1])).reshape(rho, pn, p1)
    if return_sigmas:
        return b, sigmas
    return b


def tt_round_left_orth(tt: Sequence[np.ndarray], max_rank=None, tol: float = 0.0, return_sigmas: bool = False):
    """Alg. 1's truncation loop run from the right on a left-orthogonal train
    (cores 1..d-1 have orthonormal columns in V(.), as every core of Alg. 4's
    and Alg. 2's output but the last).  Alg. 1 first orthogonalises one way
    and then truncates the other; such an input is already orthogonalised
    from the left, so the truncation runs right to left with no
    orthogonalisation pass.  Bond k: QR of H(B_k)^T = Q R, so H(B_k) = R^T Q^T;
    SVD R^T = U S W^T; keep rho columns (same rule and delta = tol ||A||_F /
    sqrt(d-1) as tt_round, ||A||_F = ||B_d||_F); B_k <- (Q W_rho)^T folded,
    B_{k-1} <- B_{k-1} x_3 (U_rho S_rho).  ``max_rank`` as in tt_round."""
    d = len(tt)
    if max_rank is None:
        caps = [None] * (d + 1)
    elif np.isscalar(max_rank):
        caps = [int(max_rank)] * (d + 1)
    else:
        caps = list(max_rank)
    b = [np.array(c, dtype=np.float64, copy=True) for c in tt]
    nrm = float(np.linalg.norm(b[d - 1]))
    delta = tol * nrm / math.sqrt(d - 1) if (tol > 0 and d > 1) else 0.0
    sigmas = [None] * (d - 1)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = b[k].shape
        q, r = _qr_pos(H(b[k]).T)              # (n r1) x r0 = Q R
        u, sg, wt = np.linalg.svd(r.T, full_matrices=False)
        rho = choose_rank(sg, delta, caps[k])
        sigmas[k - 1] = sg
        b[k] = (q @ wt[:rho, :].T).T.reshape(rho, n, r1)
        p0, pn, _ = b[k - 1].shape
        b[k - 1] = (V(b[k - 1]) @ (u[:, :rho] * sg[None, :rho])).reshape(p0, pn, rho)
    if return_sigmas:
        return b, sigmas
    return b


def tt_svd(full_tensor: np.ndarray, tol: float = 0.0, max_rank=None) -> TT:
    """TT-SVD of a full tensor (the reference the paper's quasi-numerical
    ranks are defined by, Defs. 3.2/3.3): left-to-right truncated SVDs of
    the sequential unfoldings with the same delta split as ``tt_round``."""
    shape = full_tensor.shape
    d = len(shape)
    nrm = float(np.linalg.norm(full_tensor))
    delta = tol * nrm / math.sqrt(d - 1) if (tol > 0 and d > 1) else 0.0
    cores = []
    rest = full_tensor.reshape(1, -1)
    r_prev = 1
    for k in range(d - 1):
        mat = rest.reshape(r_prev * shape[k], -1)
        u, s, vt = np.linalg.svd(mat, full_matrices=False)
        cap = None if max_rank is None else (max_rank if np.isscalar(max_rank) else max_rank[k + 1])
        rho = choose_rank(s, delta, cap)
        cores.append(u[:, :rho].reshape(r_prev, shape[k], rho))
        rest = s[:rho, None] * vt[:rho, :]
        r_prev = rho
    cores.append(rest.reshape(r_prev, shape[d - 1], 1))
    return cores
