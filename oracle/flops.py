"""Operation counts of Sec. 4 (eq. CHATT and Table 4.1).

``table41`` evaluates the paper's closed forms for uniform ranks;
``hatt1_bonds`` counts the same steps with the actual per-bond ranks
(r_k, s_k, l_k, n_k), term by term as the complexity paragraphs of Sec. 4
list them:

* HPCRL-1, per interior core: W_L costs n r s l (2r + 2s - 2), W_L W_R^T
  costs 2 n r s l^2 - r s l;
* sweep, per core: X W costs n l^2 (2 r s - 1), the Q-only econ-QR of an
  m x l matrix costs 4 m l^2 - 4 l^3 / 3, M = Q^T X costs r s l (2 l n - 1)
  and the PKP-free core update costs n r s l (2r + 2s - 2).
"""

from __future__ import annotations

from typing import Dict, Sequence


def table41(d: int, n: int, r: int, s: int, ell: int, R: int | None = None) -> Dict[str, float]:
    """Recompression cost column of Table 4.1 (uniform ranks)."""
    R = ell if R is None else R
    return {
        "tt_rounding": (d - 2) * n * (5 * r**3 * s**3 + 6 * r**2 * s**2 * ell + 2 * r * s * ell**2),
        "orthrand": (d - 2) * n * (5 * r**3 * s**3 + 2 * r**2 * s**2 * ell + 4 * r * s * ell**2),
        "randorth": (d - 2) * n * (4 * r**2 * s**2 * ell + 6 * r * s * ell**2),
        "twosided": (d - 2) * n * (6 * r**2 * s**2 * ell + 6 * r * s * ell**2),
        "hatt1": (d - 2) * (n * r * s * ell * (4 * r + 4 * s + 6 * ell)),
        "hatt2": (d - 2) * (n * r * s * (2 * r + 2 * s + 2 * ell) * (ell + R) + 2 * n * r * s * ell**2),
    }


def speedup_models(r: int, s: int, ell: int) -> Dict[str, float]:
    """SP(l) of HaTT-1 against TT-Rounding, OrthRand and RandOrth (Sec. 4)."""
    den = 4 * r * ell + 4 * s * ell + 6 * ell**2
    return {
        "tt_rounding": (5 * r**2 * s**2 + 6 * r * s * ell + 2 * ell**2) / den,
        "orthrand": (5 * r**2 * s**2 + 2 * r * s * ell + 4 * ell**2) / den,
        "randorth": (4 * r * s + 6 * ell) / (4 * r + 4 * s + 6 * ell),
    }


def hatt1_bonds(n: Sequence[int], rx: Sequence[int], ry: Sequence[int], ell: Sequence[int]) -> Dict[str, float]:
    """Per-step flop totals of HaTT-1 with actual ranks (lists of length d
    for n, d+1 for the ranks)."""
    d = len(n)
    wl = wr = xw = qr = proj = upd = 0.0
    for c in range(1, d - 1):                 # HPCRL steps on cores 2..d-1 (1-based)
        r0, r1, s0, s1 = rx[c], rx[c + 1], ry[c], ry[c + 1]
        l0, l1 = ell[c], ell[c + 1]
        wl += n[c] * l1 * (2 * s0 * s1 * r1 + 2 * s0 * r1 * r0)
        wr += 2.0 * (r0 * s0) * (n[c] * l1) * l0
    for c in range(d - 1):                    # sweep on cores 1..d-1
        l0, l1 = ell[c], ell[c + 1]
        r1, s1 = rx[c + 1], ry[c + 1]
        m = l0 * n[c]
        xw += 2.0 * m * (r1 * s1) * l1
        qr += 4.0 * m * l1 * l1 - 4.0 * l1**3 / 3.0
        proj += 2.0 * l1 * (r1 * s1) * m
        rn0, rn1, sn0, sn1 = rx[c + 1], rx[c + 2], ry[c + 1], ry[c + 2]
        upd += n[c + 1] * l1 * (2 * rn0 * sn0 * sn1 + 2 * rn0 * sn1 * rn1)
    total = wl + wr + xw + qr + proj + upd
    return {"wl": wl, "wr": wr, "xw": xw, "qr": qr, "proj": proj, "update": upd, "total": total}
