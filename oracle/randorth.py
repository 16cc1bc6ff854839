"""PartialContractionRL (eq. rtlpc) and RandOrth (Alg. 2), FP64 numpy,
applied to an explicit TT (for a Hadamard product: to its PKP cores).

Index convention in code: cores are 0-based, c = 0..d-1; bond b = 1..d-1
sits between cores b-1 and b, so the paper's W^{(k)} (an r_k s_k x l_k matrix
for the bond after core k, 1-based) is ``W[b]`` with b = k.
"""

from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .tt import H, V, _qr_pos

TT = List[np.ndarray]


def partial_contraction_rl(a: Sequence[np.ndarray], r: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Sketch matrices of eq. (partial-contraction) via the recursion of
    eq. (rtlpc): W^{(d-1)} = H(A_d) H(R_d)^T; then for k = d-1..2,
    V(B_k) = V(A_k) W^{(k)} and W^{(k-1)} = H(B_k) H(R_k)^T.
    Returns a list indexed by bond (entries 0 unused)."""
    d = len(a)
    w: List[np.ndarray] = [None] * d  # type: ignore[list-item]
    if d < 2:
        return w
    w[d - 1] = H(a[d - 1]) @ H(r[d - 1]).T
    for b in range(d - 1, 1, -1):
        c = b - 1
        r0, n, _ = a[c].shape
        t = V(a[c]) @ w[b]                                  # V(B_k)
        t = t.reshape(r0, n * w[b].shape[1])                # H(B_k)
        w[b - 1] = t @ H(r[c]).T
    return w


def randorth(a: Sequence[np.ndarray], r: Sequence[np.ndarray]) -> TT:
    """Alg. 2 with the sketch TT ``r`` (ranks l_k) given: sketch right to
    left, then for k = 1..d-1: [V(B_k), ~] = QR(B^{(k)} W^{(k)}),
    M^{(k)} = V(B_k)^T B^{(k)}, H(B_{k+1}) = M^{(k)} H(A_{k+1})."""
    d = len(a)
    if d == 1:
        return [a[0].copy()]
    w = partial_contraction_rl(a, r)
    b = [c.copy() for c in a]
    for c in range(d - 1):
        l0, n, _ = b[c].shape
        bm = V(b[c])
        q, _ = _qr_pos(bm @ w[c + 1])
        b[c] = q.reshape(l0, n, q.shape[1])
        m = q.T @ bm
        _, n1, r1 = a[c + 1].shape
        b[c + 1] = (m @ H(a[c + 1])).reshape(q.shape[1], n1, r1)
    return b
