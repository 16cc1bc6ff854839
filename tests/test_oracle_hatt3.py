"""Pins of the oracle's three-factor HaTT (x (.) y (.) w) against brute force,
RandOrth on the explicit three-way PKP cores, the two-factor oracle, and the
closed-form ranks of a trigonometric product."""

import numpy as np
import pytest

import workloads as wk
from oracle import adapt, hatt, hatt3, philox, plan, randorth, rounding, tt


def _triple(seed, n, r, s, t):
    rng = np.random.default_rng(seed)
    return (wk.gaussian_tt(rng, n, wk.feasible_ranks(n, r)), wk.gaussian_tt(rng, n, wk.feasible_ranks(n, s)),
            wk.gaussian_tt(rng, n, wk.feasible_ranks(n, t)))


def _widths(x, y, w, ell):
    n = tt.modes(x)
    ryw = [a * b for a, b in zip(tt.ranks(y), tt.ranks(w))]
    return plan.clamp_ell(n, tt.ranks(x), ryw, ell)


CASES = [
    ([4] * 5, 2, 3, 2, 7),
    ([3, 5, 2, 4], 2, 2, 3, 5),      # uneven modes and ranks
    ([6, 7], 3, 2, 2, 4),            # d = 2: no HPCRL recursion
    ([5, 6, 5], 3, 2, 3, 9),         # d = 3
    ([2] * 7, 2, 2, 2, 6),           # binary modes (the QTT shape)
    ([1, 4, 1, 3], 2, 2, 2, 3),      # modes of size 1
]


def test_pkp3_is_the_elementwise_product():
    x, y, w = _triple(1, [3, 4, 2, 3], 2, 3, 2)
    a = hatt3.pkp3(x, y, w)
    ref = tt.full(x) * tt.full(y) * tt.full(w)
    assert tt.ranks(a) == [p * q * s for p, q, s in zip(tt.ranks(x), tt.ranks(y), tt.ranks(w))]
    assert np.linalg.norm(tt.full(a) - ref) < 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,r,s,t,ell", CASES)
def test_hatt3_equals_randorth_on_explicit_pkp3(n, r, s, t, ell):
    """Three-factor HaTT is RandOrth on the three-way PKP cores with the same
    sketch: the three-mode products only rewrite the Kronecker products."""
    x, y, w = _triple(sum(n) + ell, n, r, s, t)
    l = _widths(x, y, w, ell)
    R = philox.sketch(5, n, l)
    a = hatt3.hatt3(x, y, w, R)
    b = randorth.randorth(hatt3.pkp3(x, y, w), R)
    assert tt.ranks(a) == l
    assert tt.rel_err(a, b) < 1e-12


def test_hpcrl3_equals_partial_contraction_of_explicit_cores():
    """eq. (rtlpc) on the explicit three-way PKP train gives the same sketch
    matrices as the three-mode recursion."""
    x, y, w = _triple(3, [3, 4, 3, 2, 3], 2, 2, 3)
    l = _widths(x, y, w, 6)
    R = philox.sketch(7, tt.modes(x), l)
    w3 = hatt3.hpcrl3(x, y, w, R)
    ref = randorth.partial_contraction_rl(hatt3.pkp3(x, y, w), R)
    for b in range(1, len(x)):
        assert np.allclose(w3[b], ref[b], rtol=0, atol=1e-13 * np.abs(ref[b]).max())


def test_hatt3_equals_two_factor_hatt_on_explicit_pair():
    """x (.) y (.) w = (x (.) y) (.) w: the two-factor oracle on the explicit
    PKP of x and y, with the same sketch and the same index order."""
    x, y, w = _triple(4, [4, 3, 5, 3], 2, 3, 2)
    l = _widths(x, y, w, 7)
    R = philox.sketch(8, tt.modes(x), l)
    a = hatt3.hatt3(x, y, w, R)
    b = hatt.hatt(tt.pkp(x, y), w, R)
    assert tt.rel_err(a, b) < 1e-12


def test_hatt3_exact_at_full_width():
    """With every width at its cap the output is the product itself."""
    x, y, w = _triple(5, [3, 3, 3, 3], 2, 2, 2)
    l = _widths(x, y, w, 1 << 20)
    a = hatt3.hatt3(x, y, w, philox.sketch(9, tt.modes(x), l))
    ref = tt.full(x) * tt.full(y) * tt.full(w)
    assert np.linalg.norm(tt.full(a) - ref) < 1e-12 * np.linalg.norm(ref)


def test_hatt3_left_orthogonal_projection():
    """Cores 1..d-1 are left-orthogonal and the output is an orthogonal
    projection of the product: ||z||^2 = ||X||^2 + ||z - X||^2."""
    x, y, w = _triple(6, [4, 4, 4, 4], 2, 2, 2)
    l = _widths(x, y, w, 4)
    a = hatt3.hatt3(x, y, w, philox.sketch(10, tt.modes(x), l))
    for c in range(len(a) - 1):
        v = tt.V(a[c])
        assert np.allclose(v.T @ v, np.eye(v.shape[1]), atol=1e-13)
    fz = tt.full(x) * tt.full(y) * tt.full(w)
    fa = tt.full(a)
    lhs = np.linalg.norm(fz) ** 2
    rhs = np.linalg.norm(fa) ** 2 + np.linalg.norm(fz - fa) ** 2
    assert abs(lhs - rhs) < 1e-12 * lhs
    assert np.linalg.norm(fz - fa) > 1e-3 * np.linalg.norm(fz)


def test_hatt3_trig_cube_closed_form_ranks():
    """u of rank 2J (cos, sin of frequencies 1..J per mode): u^3 spans the
    frequencies 0..3J, so its TT ranks are 6J + 1 (J = 3: 19), which the
    truncated three-factor HaTT finds at tol 1e-10 with the error in bound."""
    u = wk.trig_u(2, n=32, terms=6, nfreq=3)
    n = tt.modes(u)
    l = plan.clamp_ell(n, tt.ranks(u), [a * a for a in tt.ranks(u)], 30)
    a = rounding.tt_round_left_orth(hatt3.hatt3(u, u, u, philox.sketch(3, n, l)), tol=1e-10)
    assert tt.ranks(a) == [1, 19, 19, 1]
    ref = tt.full(u) ** 3
    assert np.linalg.norm(tt.full(a) - ref) < 1e-10 * np.linalg.norm(ref)


def test_adaptive_triple_reaches_tolerance():
    """The tolerance rule with a triple: converged, ranks 6J + 1, error <= tol."""
    u = wk.trig_u(4, n=32, terms=6, nfreq=3)
    outs, l, attempts, ok = adapt.hatt_adaptive([(u, u, u)], tol=1e-9, seed=1)
    assert ok
    assert tt.ranks(outs[0]) == [1, 19, 19, 1]
    ref = tt.full(u) ** 3
    assert np.linalg.norm(tt.full(outs[0]) - ref) < 1e-9 * np.linalg.norm(ref)
