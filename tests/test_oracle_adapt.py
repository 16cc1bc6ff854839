"""Pins of the tolerance-driven (adaptive width) oracle on the trig workload
shape, where the ranks of the products are known in closed form: products of
sin/cos of frequencies <= F span {1, cos mx, sin mx : m <= 2F} (rank 4F+1) and,
for a triple product, frequencies <= 3F (rank 6F+1)."""

import numpy as np
import pytest

import workloads as wk
from oracle import adapt, plan, rounding, tt


@pytest.fixture(scope="module")
def small_trig():
    return wk.trig_u(3, n=48, terms=12, nfreq=6)


def test_trig_input_ranks_and_values(small_trig):
    u = small_trig
    assert tt.ranks(u) == [1, 12, 12, 1]
    f = tt.full(u)
    assert f.shape == (48, 48, 48)
    # u is a sum of 12 separable terms: every unfolding has rank 12
    assert np.linalg.matrix_rank(f.reshape(48, -1), tol=1e-10 * np.abs(f).max()) == 12


def test_product_ranks_closed_form(small_trig):
    u = small_trig
    u2 = tt.pkp(u, u)
    r2 = rounding.tt_round(u2, tol=1e-12)
    assert tt.ranks(r2) == [1, 25, 25, 1]
    u3 = rounding.tt_round(tt.pkp(r2, u), tol=1e-12)
    assert tt.ranks(u3) == [1, 37, 37, 1]
    fu = tt.full(u)
    assert np.linalg.norm(tt.full(u3) - fu ** 3) <= 1e-10 * np.linalg.norm(fu ** 3)


def test_adaptive_meets_tolerance_and_finds_rank(small_trig):
    u = small_trig
    tol = 1e-8
    outs, ell, attempts, ok = adapt.hatt_adaptive([(u, u)], tol=tol, seed=5)
    assert ok and attempts >= 2            # 12 + 8 = 20 < 25 forces growth
    x = outs[0]
    assert tt.ranks(x) == [1, 25, 25, 1]
    fu = tt.full(u)
    err = np.linalg.norm(tt.full(x) - fu ** 2) / np.linalg.norm(fu ** 2)
    assert err <= tol
    # acceptance rule: slack on every bond or the bond at its largest width
    cap = plan.clamp_ell(tt.modes(u), tt.ranks(u), tt.ranks(u), adapt.BIG)
    for k in (1, 2):
        assert tt.ranks(x)[k] <= ell[k] - 8 or ell[k] == cap[k]


def test_adaptive_growth_rule():
    cap = [1, 50, 300, 1]
    assert adapt.grow([1, 20, 40, 1], [2], cap) == [1, 20, 68, 1]
    assert adapt.grow([1, 48, 40, 1], [1, 2], cap) == [1, 50, 68, 1]
    assert adapt.failing_bonds([[1, 12, 30, 1], [1, 5, 33, 1]], [1, 20, 40, 1], cap) == [2]
    assert adapt.failing_bonds([[1, 50, 5, 1]], [1, 50, 40, 1], cap) == []
