"""Tolerance-driven HaTT: grow the sketch widths until the truncation leaves
slack (oracle side).

The paper fixes target ranks and leaves tolerance control to future work
(Sec. 6); it notes that when the smallest singular value of a sketch is not
small enough, l should be increased (Sec. 5.1.1).  The rule implemented here
(the same on both sides):

* start: l_k = max(r_k, s_k) + p (p = oversampling, default 8), clamped;
* run HaTT with the sketch keyed by seed + attempt, then truncate at
  tol sqrt(3) / 2 (Alg. 1's truncation loop from the right on HaTT's
  left-orthogonal output, rounding.tt_round_left_orth);
* accept when every bond keeps rho_k <= l_k - p, or l_k already equals its
  largest feasible value (then the sketch captured the bond exactly), and
  the sketch captured z's range to within tol / 2: the untruncated HaTT
  result X is an orthogonal projection of z, so ||z - X||^2 =
  ||z||^2 - ||X||^2, and the truncation's error is orthogonal to it, so the
  two shares add up to at most tol (the capture test cannot resolve
  ||z - X||^2 below 256 eps ||z||^2, its floor);
* otherwise grow l_k = min(cap_k, ceil(1.5 l_k) + p) on each bond failing
  the slack test, or on every bond below its cap when only the capture test
  failed, and retry; give up after ``max_attempts``.

For a batch of pairs the widths are common to all pairs and a bond fails if
it fails for any pair.  A triple (x, y, w) in place of a pair runs the
three-factor HaTT (hatt3) under the slack rule alone (truncation at tol, no
capture test), with r_k s_k t_k as the product rank in the clamps and
max(r_k, s_k, t_k) + p as the start.
"""

from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from . import philox, plan, rounding, tt
from .hatt import hatt
from .hatt3 import hatt3

BIG = 1 << 40
TRUNC_SHARE = math.sqrt(3.0) / 2.0
CAPTURE_SHARE2 = 0.25
CAPTURE_FLOOR = 256.0 * np.finfo(np.float64).eps


def initial_widths(n, rx, ry, p: int = 8) -> List[int]:
    d = len(n)
    req = [1] + [max(int(rx[k]), int(ry[k])) + p for k in range(1, d)] + [1]
    return plan.clamp_ell(n, rx, ry, req)


def grow(ell: Sequence[int], fail: Sequence[int], cap: Sequence[int], p: int = 8) -> List[int]:
    out = list(ell)
    for k in fail:
        out[k] = min(int(cap[k]), int(math.ceil(1.5 * ell[k])) + p)
    return out


def failing_bonds(kept: Sequence[Sequence[int]], ell: Sequence[int], cap: Sequence[int], p: int = 8) -> List[int]:
    d = len(ell) - 1
    bad = set()
    for rho in kept:
        for k in range(1, d):
            if rho[k] > ell[k] - p and ell[k] < cap[k]:
                bad.add(k)
    return sorted(bad)


def hatt_adaptive(pairs, tol: float, seed: int, p: int = 8, max_attempts: int = 8, variant: int = 1,
                  ep: float = 0.0, ell0: Sequence[int] | None = None, seed_step: int = 1):
    """``pairs``: list of (y, z) of one shape.  Attempt a uses the sketch
    keyed by seed + a * seed_step; ``ell0`` replaces the starting widths
    (a predicted start).  Returns (outputs, widths used, attempts,
    converged)."""
    ops0 = pairs[0]
    n = tt.modes(ops0[0])
    rk = [tt.ranks(o) for o in ops0]
    rx = rk[0]
    ry = [int(np.prod([r[k] for r in rk[1:]])) for k in range(len(rx))]
    cap = plan.clamp_ell(n, rx, ry, BIG)
    if ell0 is None:
        req = [1] + [max(r[k] for r in rk) + p for k in range(1, len(n))] + [1]
        ell = plan.clamp_ell(n, rx, ry, req)
    else:
        ell = list(ell0)
    two = len(ops0) == 2 and len(n) >= 2
    z2 = [tt.norm(tt.pkp(ops[0], ops[1])) ** 2 for ops in pairs] if two else None
    outs = None
    for attempt in range(max_attempts):
        l = plan.clamp_ell(n, rx, ry, ell)
        R = philox.sketch(seed + attempt * seed_step, n, l)
        raws = [hatt(ops[0], ops[1], R, variant, ep) if len(ops) == 2 else hatt3(ops[0], ops[1], ops[2], R)
                for ops in pairs]
        outs = [rounding.tt_round_left_orth(x, tol=tol * TRUNC_SHARE if two else tol) for x in raws]
        bad = failing_bonds([tt.ranks(o) for o in outs], l, cap, p)
        if two and not bad:
            for x, zz in zip(raws, z2):
                c2 = max(0.0, zz - tt.norm(x) ** 2)
                if c2 > max(CAPTURE_SHARE2 * tol * tol, CAPTURE_FLOOR) * zz:
                    bad = [k for k in range(1, len(n)) if l[k] < cap[k]]
                    break
        if not bad:
            return outs, l, attempt + 1, True
        ell = grow(l, bad, cap, p)
    return outs, l, max_attempts, False
