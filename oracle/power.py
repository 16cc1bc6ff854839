"""Power iteration for the largest entry of a TT tensor Y (Sec. 5,
Example 3), each step's Hadamard product recompressed by HaTT.  FP64
numpy; test infrastructure (see the package header).

Reading (the paper names the method and its settings, not its formulas):
starting from the all-ones tensor X_0 normalised to unit Frobenius norm,
step t computes Z_t = HaTT(X_t (.) Y) at sketch width l with the Philox
sketch keyed by seed + t (no truncation: the output rank is l), the
estimate lambda_t = ||Z_t||_F (= ||Y (.) X_t|| / ||X_t|| up to the
recompression error), and X_{t+1} = Z_t / lambda_t.  For Y >= 0, lambda_t
tends to max(Y) as X_t concentrates on the largest entry (the power method
for the diagonal operator of Y).
"""

from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import hatt as ohatt
from . import philox, plan, tt

TT = List[np.ndarray]


def ones_tt(n: Sequence[int]) -> TT:
    """The all-ones tensor as a rank-1 TT."""
    return [np.ones((1, k, 1)) for k in n]


def power_iteration(y: Sequence[np.ndarray], ell: int, iters: int, seed: int) -> Tuple[List[float], TT]:
    n = tt.modes(y)
    x = ones_tt(n)
    x[0] = x[0] / tt.norm(x)
    lam: List[float] = []
    for t in range(iters):
        widths = plan.clamp_ell(n, tt.ranks(x), tt.ranks(y), ell)
        z = ohatt.hatt(x, y, philox.sketch(seed + t, n, widths))
        nz = tt.norm(z)
        lam.append(nz)
        z[0] = z[0] / nz
        x = z
    return lam, x
