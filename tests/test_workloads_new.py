"""Pins of the power-iteration and QTT input generators against their closed
forms (CPU): the rank-d TT of a separable sum equals the sum on the full
grid, and the QTT trig field equals sum_t a_t prod_m sin(k_tm x_m)."""

import math

import numpy as np

import workloads as wk
from oracle import tt


def test_separable_sum_tt_matches_full_grid():
    for vals in (wk.qing_values(5, n=4), wk.alpine_values(4, n=5)):
        cores = wk.separable_sum_tt(vals)
        d = len(vals)
        assert tt.ranks(cores) == [1] + [d] * (d - 1) + [1]
        grids = np.meshgrid(*vals, indexing="ij")
        assert np.allclose(tt.full(cores).reshape(-1), sum(grids).reshape(-1), rtol=1e-13, atol=0)


def test_qing_and_alpine_maxima_are_at_the_grid_ends():
    """The largest Qing entry sits at x_i = -500 (farthest from i), i.e.
    sum_i (500 + i)^2; the Alpine maximum is d times the largest per-mode
    value, which the grid's endpoints +-2.5 pi attain."""
    d = 6
    q = wk.qing_values(d)
    assert math.isclose(sum(v.max() for v in q), sum((500 + i) ** 2 for i in range(1, d + 1)), rel_tol=1e-15)
    a = wk.alpine_values(d)
    x = 2.5 * math.pi
    assert math.isclose(a[0].max(), abs(x * math.sin(x) + 0.1 * x), rel_tol=1e-14)


def test_qtt_sine_and_field_match_closed_form():
    D = 4
    n = 1 << D
    h = 2 * math.pi / n
    x = h * (np.arange(n) + 0.5)
    for k in (1.0, 3.0):
        s = wk.qtt_sine(k, D)
        assert tt.ranks(s) == [1] + [2] * (D - 1) + [1]
        assert np.allclose(tt.full(s).reshape(-1), np.sin(k * x), atol=1e-14)
    cores, a, ks = wk.qtt_trig_field(5, D, terms=4)
    assert max(tt.ranks(cores)) <= 8
    f = np.zeros((n, n, n))
    for t in range(4):
        f += a[t] * np.einsum("i,j,k->ijk", *[np.sin(ks[t, m] * x) for m in range(3)])
    assert np.allclose(tt.full(cores).reshape(-1), f.reshape(-1), atol=1e-13)


def test_oracle_power_iteration_exact_and_converging():
    """With sketches as wide as the products' ranks, each HaTT step is exact
    and the oracle's estimates equal ||Y^(t+1)|| / ||Y^t|| on the full
    tensor (Hadamard powers); at the paper's width l = 5 the estimates rise
    toward the largest entry, known in closed form (Qing: x_i = -500 in
    every mode; Alpine: d times the largest per-mode value)."""
    from oracle import power
    vals = wk.qing_values(4, n=5)
    y = wk.separable_sum_tt(vals)
    fy = tt.full(y).reshape(-1)
    lam, x = power.power_iteration(y, ell=10 ** 6, iters=8, seed=3)
    for t, lt in enumerate(lam):
        exact = np.linalg.norm(fy ** (t + 1)) / np.linalg.norm(fy ** t)
        assert abs(lt - exact) <= 1e-12 * exact
    for vals in (wk.qing_values(5, n=6), wk.alpine_values(5, n=6)):
        y = wk.separable_sum_tt(vals)
        lam, x = power.power_iteration(y, ell=5, iters=60, seed=3)
        top = sum(v.max() for v in vals)
        assert abs(lam[-1] - top) <= 1e-2 * top
        assert lam[-1] > lam[10] > lam[0]
        assert abs(tt.norm(x) - 1.0) <= 1e-12
