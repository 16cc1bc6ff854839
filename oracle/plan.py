"""Sketch-width clamps applied before a recompression (oracle side).

The paper assumes max(r, s) <~ l << r s (Sec. 2.2) and fixes target ranks;
it does not say what happens when a requested width cannot be realised.  The
reading used on both sides:

* l_0 = l_d = 1;
* l_k <= r_k s_k (the rank of the Hadamard product at bond k, Sec. 2.2);
* l_k <= l_{k-1} n_k, left to right: the sketched frame of Alg. 4 is an
  (l_{k-1} n_k) x l_k matrix and its economy QR needs rows >= columns
  (Sec. 4, econ-QR of an m x n matrix with m > n);
* l_{k-1} <= n_k l_k, right to left: the same for the right-to-left QR of
  Alg. 1 applied afterwards.
"""

from __future__ import annotations

from typing import List, Sequence


def clamp_ell(n: Sequence[int], rx: Sequence[int], ry: Sequence[int], ell) -> List[int]:
    d = len(n)
    if isinstance(ell, int):
        req = [ell] * (d + 1)
    else:
        req = list(ell)
        if len(req) != d + 1:
            raise ValueError("ell must have d+1 entries")
    out = [1] * (d + 1)
    for k in range(1, d):
        out[k] = max(1, min(int(req[k]), int(rx[k]) * int(ry[k])))
    for k in range(1, d):
        out[k] = min(out[k], out[k - 1] * int(n[k - 1]))
    for k in range(d - 1, 0, -1):
        out[k] = min(out[k], int(n[k]) * out[k + 1])
    return out
