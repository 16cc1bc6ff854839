"""Learned per-bond width predictor (oracle side, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper picks sketch widths by hand and suggests growing l when a sketch
is too narrow (Sec. 5.1.1); tolerance control is left open (Sec. 6).  The
adaptive rule of ``adapt`` answers that by retrying with wider sketches.
This module is the plain definition of a small regression network that
predicts, per bond, the rank the truncation keeps and the width the
adaptive rule would accept, from cheap statistics of the two input cores,
so that a recompression can start at (nearly) the right width:

* ``features``      21 inputs per bond k = 1..d-1 of a pair (x, y);
* ``labels``        targets from an accepted adaptive recompression;
* ``forward`` / ``loss_and_grad`` / ``adam``   a 21-128-128-2 tanh MLP,
                    mean squared error in standardised label units, and the
                    Adam update of Kingma and Ba (ICLR 2015, Algorithm 1);
* ``fit_stats``     standardisation of inputs and targets;
* ``widths``        predicted widths, clamped like every other width.

Layouts (shared with the HIP library by specification, not by code):

theta (trained, 19586 values)   W1[128][21] b1[128] W2[128][128] b2[128]
                                W3[2][128] b3[2], row-major, in that order;
stats (46 values)               mu_x[21] sd_x[21] mu_y[2] sd_y[2].

Feature row of bond k (1-based; core index k-1):
  0 ln r_k(x)   1 ln r_k(y)   2 ln n_k   3 k/d   4 ln d
  5..12  quantiles at j/7 (j = 0..7, linear interpolation between order
         statistics) of ln max(c_a, 1e-300), c_a = sum_{b,i} x_k[b, i, a]^2,
         the diagonal of V(x_k)^T V(x_k);
  13..20 the same for y.
Target row: ln rho_k, ln l*_k with l*_k = min(cap_k, rho_k + p), the
narrowest width the acceptance rule takes for the kept rank rho_k.
"""

from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

from . import plan

N_IN, N_H, N_OUT = 21, 128, 2
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_THETA = sum(int(np.prod(s)) for _, s in SIZES)
N_STATS = 2 * N_IN + 2 * N_OUT
LOG_FLOOR = 1e-300


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SIZES:
        sz = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def quantiles8(v: Sequence[float]) -> List[float]:
    """Values at q = j/7, j = 0..7: sorted v, position h = (len - 1) q,
    linear interpolation between the two order statistics around h."""
    s = sorted(float(t) for t in v)
    r = len(s)
    out = []
    for j in range(8):
        h = (r - 1) * (j / 7.0)
        lo = int(math.floor(h))
        hi = min(lo + 1, r - 1)
        out.append(s[lo] + (h - lo) * (s[hi] - s[lo]))
    return out


def log_col_norms(core: np.ndarray) -> List[float]:
    """ln of the squared column norms of the left unfolding V(core)."""
    rp, n, rn = core.shape
    v = core.reshape(rp * n, rn)
    out = []
    for a in range(rn):
        c = 0.0
        for t in range(rp * n):
            c += float(v[t, a]) * float(v[t, a])
        out.append(math.log(max(c, LOG_FLOOR)))
    return out


def features(x: Sequence[np.ndarray], y: Sequence[np.ndarray]) -> np.ndarray:
    """(d-1) x 21 feature rows of the bonds of one pair."""
    d = len(x)
    rows = []
    for k in range(1, d):
        cx, cy = x[k - 1], y[k - 1]
        row = [math.log(cx.shape[2]), math.log(cy.shape[2]), math.log(cx.shape[1]), k / d, math.log(d)]
        row += quantiles8(log_col_norms(cx))
        row += quantiles8(log_col_norms(cy))
        rows.append(row)
    return np.array(rows, dtype=np.float64).reshape(d - 1, N_IN)


def labels(kept: Sequence[int], cap: Sequence[int], p: int = 8) -> np.ndarray:
    """(d-1) x 2 targets from the kept ranks of an accepted recompression."""
    d = len(kept) - 1
    return np.array([[math.log(kept[k]), math.log(min(int(cap[k]), int(kept[k]) + p))] for k in range(1, d)],
                    dtype=np.float64).reshape(d - 1, N_OUT)


def fit_stats(feat: np.ndarray, lab: np.ndarray) -> np.ndarray:
    """Column means and population standard deviations (a deviation below
    1e-8 is replaced by 1, so constant columns pass through centred)."""
    def ms(a):
        mu = a.mean(axis=0)
        sd = np.sqrt(((a - mu) ** 2).mean(axis=0))
        sd = np.where(sd < 1e-8, 1.0, sd)
        return mu, sd
    mx, sx = ms(np.asarray(feat, dtype=np.float64))
    my, sy = ms(np.asarray(lab, dtype=np.float64))
    return np.concatenate([mx, sx, my, sy])


def _split_stats(stats):
    s = np.asarray(stats, dtype=np.float64)
    return s[:N_IN], s[N_IN:2 * N_IN], s[2 * N_IN:2 * N_IN + N_OUT], s[2 * N_IN + N_OUT:]


def forward(theta, stats, feat):
    """Standardised outputs o (rows x 2) and the cached activations."""
    P = unpack(theta)
    mx, sx, _, _ = _split_stats(stats)
    xh = (np.asarray(feat, dtype=np.float64) - mx) / sx
    h1 = np.tanh(xh @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    o = h2 @ P["W3"].T + P["b3"]
    return o, (xh, h1, h2)


def predict(theta, stats, feat) -> np.ndarray:
    """Predictions in target units (ln rho, ln l*)."""
    o, _ = forward(theta, stats, feat)
    _, _, my, sy = _split_stats(stats)
    return o * sy + my


def loss_and_grad(theta, stats, feat, lab):
    """L = 1/(2B) sum_b sum_o (o_bo - t_bo)^2, t = standardised targets;
    returns (L, dL/dtheta packed like theta)."""
    P = unpack(theta)
    _, _, my, sy = _split_stats(stats)
    o, (xh, h1, h2) = forward(theta, stats, feat)
    t = (np.asarray(lab, dtype=np.float64) - my) / sy
    B = o.shape[0]
    diff = o - t
    L = 0.5 * float((diff ** 2).sum()) / B
    d3 = diff / B
    g = {"W3": d3.T @ h2, "b3": d3.sum(axis=0)}
    d2 = (d3 @ P["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ xh
    g["b1"] = d1.sum(axis=0)
    return L, pack(g)


def adam(theta, m, v, grad, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * grad
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return np.asarray(theta, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def widths(pred: np.ndarray, n: Sequence[int], rx: Sequence[int], ry: Sequence[int], margin: float,
           p: int = 8):
    """Widths and predicted kept ranks of one pair from its (d-1) x 2
    prediction rows: l_k = ceil((1 + margin) max(e^{pred_k,1},
    e^{pred_k,0} + p)), rho_k = ceil(e^{pred_k,0}), then the usual clamps."""
    d = len(n)
    ell, rho = [1] * (d + 1), [1] * (d + 1)
    for k in range(1, d):
        a, b = float(pred[k - 1][0]), float(pred[k - 1][1])
        w = max(math.exp(b), math.exp(a) + p)
        ell[k] = max(1, int(math.ceil((1.0 + margin) * w)))
        rho[k] = max(1, int(math.ceil(math.exp(a))))
    return plan.clamp_ell(n, rx, ry, ell), rho
