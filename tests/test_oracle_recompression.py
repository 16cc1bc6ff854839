"""Pins of the oracle's recompression routines (Alg. 1-4) against brute
force, theorem inequalities, invariants and exact special cases."""

import math

import numpy as np
import pytest

import workloads as wk
from oracle import adapt, hatt, philox, plan, randorth, rounding, tt


def _setup(y, z, ell, seed=11):
    n, rx, ry = tt.modes(y), tt.ranks(y), tt.ranks(z)
    l = plan.clamp_ell(n, rx, ry, ell)
    return l, philox.sketch(seed, n, l)


def _rand_pair(seed, n, r, s):
    rng = np.random.default_rng(seed)
    rx, ry = wk.feasible_ranks(n, r), wk.feasible_ranks(n, s)
    return wk.gaussian_tt(rng, n, rx), wk.gaussian_tt(rng, n, ry)


CASES = [
    ([4] * 6, 3, 3, 9),
    ([4] * 6, 3, 3, 4),
    ([3, 5, 2, 4, 3], 2, 4, 5),       # r != s, uneven modes
    ([6, 7], 3, 2, 4),                # d = 2: empty HPCRL loop
    ([5, 6, 5], 4, 3, 7),             # d = 3
    ([2] * 8, 2, 3, 5),               # binary modes
    ([1, 4, 1, 3], 2, 2, 3),          # modes of size 1
]


@pytest.mark.parametrize("n,r,s,ell", CASES)
def test_hatt_equals_randorth_on_explicit_pkp(n, r, s, ell):
    """HaTT-1 is RandOrth applied to the PKP cores with the same sketch
    (the algebra of Sec. 3.1 and eq. M*core0 only rewrites the products)."""
    y, z = _rand_pair(sum(n) + ell, n, r, s)
    l, R = _setup(y, z, ell)
    x1 = hatt.hatt(y, z, R)
    x2 = randorth.randorth(tt.pkp(y, z), R)
    assert tt.ranks(x1) == l
    assert tt.rel_err(x1, x2) < 1e-13


def test_hpcrl_sketches_equal_definition_bruteforce():
    """eq. (partial-contraction): W^{(k)} = H(A_{k+1:d}) H(R_{k+1:d})^T, with
    the partial products formed explicitly from full sub-trains."""
    y, z = _rand_pair(21, [3, 4, 3, 2, 3], 2, 3)
    l, R = _setup(y, z, 5)
    a = tt.pkp(y, z)
    w = hatt.hpcrl(y, z, R)
    d = len(a)
    for b in range(1, d):
        # H(A_{b+1:d}): rows = left rank of core b (0-based), columns = all trailing modes
        ha = a[b].reshape(a[b].shape[0], -1)
        hr = R[b].reshape(R[b].shape[0], -1)
        for c in range(b + 1, d):
            ha = (ha.reshape(-1, a[c].shape[0]) @ tt.H(a[c])).reshape(ha.shape[0], -1)
            hr = (hr.reshape(-1, R[c].shape[0]) @ tt.H(R[c])).reshape(hr.shape[0], -1)
        ref = ha @ hr.T
        assert np.allclose(w[b], ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    w2 = randorth.partial_contraction_rl(a, R)
    for b in range(1, d):
        assert np.allclose(w[b], w2[b], rtol=0, atol=1e-13 * np.abs(w2[b]).max())


def test_exact_rank_reproduces_product_bruteforce():
    """Tiny workload, exact rank 9 (clamped [1,4,9,9,9,4,1]): the output is
    the Hadamard product itself; its TT-SVD ranks are the clamped ranks."""
    y, z = wk.tiny_pair(0)
    l, R = _setup(y, z, 9)
    assert l == [1, 4, 9, 9, 9, 4, 1]
    x = hatt.hatt(y, z, R)
    fz = tt.full(y) * tt.full(z)
    assert np.linalg.norm(tt.full(x) - fz) < 1e-13 * np.linalg.norm(fz)
    assert tt.ranks(rounding.tt_svd(fz, tol=1e-13)) == [1, 4, 9, 9, 9, 4, 1]


def test_projection_property_and_left_orthogonality():
    """The output is an orthogonal projection of y (.) z: cores 1..d-1 are
    left-orthogonal and ||z||^2 = ||X||^2 + ||z - X||^2."""
    y, z = wk.tiny_pair(1)
    l, R = _setup(y, z, 4)
    x = hatt.hatt(y, z, R)
    for c in range(len(x) - 1):
        v = tt.V(x[c])
        assert np.allclose(v.T @ v, np.eye(v.shape[1]), atol=1e-13)
    fz = tt.full(y) * tt.full(z)
    fx = tt.full(x)
    lhs = np.linalg.norm(fz) ** 2
    rhs = np.linalg.norm(fx) ** 2 + np.linalg.norm(fz - fx) ** 2
    assert abs(lhs - rhs) < 1e-12 * lhs
    assert np.linalg.norm(fz - fx) > 1e-3 * np.linalg.norm(fz)   # really truncated


def test_sketch_rank_bounded_by_separation_rank():
    """Thm. 3.1: rank W^{(k)} <= separation rank.  For z = y (.) y the
    product's unfoldings have rank <= r (r+1)/2 = 6 < r^2 = 9."""
    y, _ = wk.tiny_pair(2)
    l, R = _setup(y, y, 9)
    w = hatt.hpcrl(y, y, R)
    fz = tt.full(y) ** 2
    shape = fz.shape
    for b in range(1, len(y)):
        unf = fz.reshape(int(np.prod(shape[:b])), -1)
        sep = np.linalg.matrix_rank(unf, tol=1e-12 * np.linalg.norm(unf, 2))
        rk = np.linalg.matrix_rank(w[b], tol=1e-12 * np.linalg.norm(w[b], 2))
        assert sep <= 6
        assert rk <= sep


def test_round_matches_tt_svd_of_full_tensor():
    """Alg. 1 with tolerance reproduces TT-SVD of the full tensor (same ranks,
    same tensor) and meets the error bound ||A - B|| <= tol ||A||."""
    y, z = wk.tiny_pair(5)
    a = tt.pkp(y, z)
    fz = tt.full(a)
    for tol in (1e-1, 3e-2, 1e-3):
        b = rounding.tt_round(a, tol=tol)
        c = rounding.tt_svd(fz, tol=tol)
        assert tt.ranks(b) == tt.ranks(c)
        err = np.linalg.norm(tt.full(b) - fz) / np.linalg.norm(fz)
        assert err <= tol * (1 + 1e-12)
        assert np.linalg.norm(tt.full(b) - tt.full(c)) < 1e-10 * np.linalg.norm(fz)
    b = rounding.tt_round(a, max_rank=4)
    c = rounding.tt_svd(fz, max_rank=4)
    assert max(tt.ranks(b)) == 4
    assert np.linalg.norm(tt.full(b) - tt.full(c)) < 1e-10 * np.linalg.norm(fz)


def test_round_truncation_lower_bound_lemma33():
    """Lemma 3.3: for a left-orthogonal A and its TT-SVD B at absolute error
    eps, ||A - B||^2 >= sum_k sigma^2_{r_k+1}(H(A_{k+1:d}))."""
    y, z = wk.tiny_pair(6)
    a = tt.orthogonalize_lr(tt.pkp(y, z))
    fa = tt.full(a)
    b = rounding.tt_svd(fa, max_rank=3)
    rb = tt.ranks(b)
    err2 = np.linalg.norm(tt.full(b) - fa) ** 2
    bound = 0.0
    d = len(a)
    for k in range(1, d):
        h = a[k].reshape(a[k].shape[0], -1)
        for c in range(k + 1, d):
            h = (h.reshape(-1, a[c].shape[0]) @ tt.H(a[c])).reshape(h.shape[0], -1)
        sv = np.linalg.svd(h, compute_uv=False)
        if rb[k] < len(sv):
            bound += sv[rb[k]] ** 2
    assert err2 >= bound * (1 - 1e-12)
    assert bound > 0


def test_truncated_special_case_is_sketch_independent():
    """Exact-rank HaTT followed by Alg. 1 at rank 4 equals Alg. 1 at rank 4
    on the explicit product; HaTT at l=4 is no better than that."""
    y, z = wk.tiny_pair(7)
    a = tt.pkp(y, z)
    ref = rounding.tt_round(a, max_rank=4)
    for seed in (1, 2):
        l, R = _setup(y, z, 9, seed)
        got = rounding.tt_round(hatt.hatt(y, z, R), max_rank=4)
        assert tt.rel_err(got, ref) < 1e-12
    l4, R4 = _setup(y, z, 4, 3)
    assert tt.rel_err(hatt.hatt(y, z, R4), a) >= tt.rel_err(ref, a) * (1 - 1e-12)


def test_sketch_scale_and_gauge_invariance():
    """Only range(X W) enters the QR of Alg. 4, so rescaling the sketch or a
    gauge change R_k <- G_{k-1}^{-1} R_k G_k leaves the output unchanged."""
    y, z = _rand_pair(8, [4, 5, 4, 5, 4], 3, 2)
    l, R = _setup(y, z, 4)
    x0 = hatt.hatt(y, z, R)
    xs = hatt.hatt(y, z, [3.7 * c for c in R])
    assert tt.rel_err(xs, x0) < 1e-12
    rng = np.random.default_rng(0)
    G = [np.eye(1)] + [rng.standard_normal((l[k], l[k])) + 3 * np.eye(l[k]) for k in range(1, len(y))] + [np.eye(1)]
    Rg = []
    for k, c in enumerate(R):
        Rg.append(np.einsum("ab,bic,cd->aid", np.linalg.inv(G[k]), c, G[k + 1]))
    assert tt.rel_err(hatt.hatt(y, z, Rg), x0) < 1e-11


def test_hatt2_reduces_to_hatt1_and_truncates_terms():
    """HaTT-2 with ep -> 0 keeps all terms and equals HaTT-1; a large ep keeps
    fewer rank-1 terms (sigma > ep ||W||_2)."""
    y, z = _rand_pair(9, [4, 5, 4, 5, 4], 3, 3)
    l, R = _setup(y, z, 6)
    x1 = hatt.hatt(y, z, R, variant=1)
    x2 = hatt.hatt(y, z, R, variant=2, ep=1e-15)
    assert tt.rel_err(x2, x1) < 1e-12
    w, used = hatt.hpcrl(y, z, R, variant=2, ep=0.3, return_split_ranks=True)
    for b in range(2, len(y)):
        wfull = hatt.hpcrl(y, z, R, variant=1)[b]
        sv = np.linalg.svd(wfull, compute_uv=False)
        assert used[b] == max(1, int(np.sum(sv > 0.3 * sv[0])))


def test_order_one_and_two():
    rng = np.random.default_rng(10)
    y = [rng.standard_normal((1, 7, 1))]
    z = [rng.standard_normal((1, 7, 1))]
    x = hatt.hatt(y, z, philox.sketch(1, [7], [1, 1]))
    assert np.allclose(x[0][0, :, 0], y[0][0, :, 0] * z[0][0, :, 0])
    y, z = _rand_pair(11, [6, 7], 3, 2)
    l, R = _setup(y, z, 6)
    assert l == [1, 6, 1]
    x = hatt.hatt(y, z, R)
    fz = tt.full(y) * tt.full(z)
    assert np.linalg.norm(tt.full(x) - fz) < 1e-13 * np.linalg.norm(fz)


def _reversed_full(a):
    """Full tensor with its modes in reverse order."""
    f = tt.full(a)
    return np.transpose(f, tuple(range(f.ndim - 1, -1, -1)))


def _reverse_train(cores):
    return [np.transpose(c, (2, 1, 0)) for c in reversed(cores)]


@pytest.mark.parametrize("cap,tol", [(None, 1e-12), (3, 0.0), ([None, 2, 5, 4, 3, None], 0.0), (None, 0.2)])
def test_round_left_orth_equals_reverse_tt_svd(cap, tol):
    """The right-to-left truncation of a left-orthogonal train equals TT-SVD
    of the full tensor run from the last mode (the TT-SVD of the
    mode-reversed tensor, reversed back): same ranks, same tensor.  The
    train is a random one made left-orthogonal, so only the tensor, not
    the gauge, is shared with the reference."""
    rng = np.random.default_rng(11)
    n = [3, 4, 3, 5, 2]
    a = [rng.standard_normal((r0, m, r1)) for r0, m, r1 in zip([1, 3, 6, 6, 4], n, [3, 6, 6, 4, 1])]
    a = tt.orthogonalize_lr(a)
    got = rounding.tt_round_left_orth(a, max_rank=cap, tol=tol)
    rcap = None if cap is None or np.isscalar(cap) else list(reversed(cap))
    ref = _reverse_train(rounding.tt_svd(_reversed_full(a), tol=tol, max_rank=cap if np.isscalar(cap) else rcap))
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= 1e-12
    if cap is None:
        full = tt.full(a)
        assert np.linalg.norm(tt.full(got) - full) <= max(tol, 1e-13) * np.linalg.norm(full) * (1 + 1e-12)


def test_round_left_orth_on_hatt_output():
    """Alg. 4's output is left-orthogonal: the right-to-left truncation
    without an orthogonalisation pass keeps the Alg. 1 error guarantee
    (within tol of the untruncated result) and, in the exact-rank regime,
    gives the same tensor and ranks as Alg. 1."""
    y, z = wk.spectral_pair(6, 6, 8, 6, 5)
    l = plan.clamp_ell(tt.modes(y), tt.ranks(y), tt.ranks(z), [1] + [24] * 5 + [1])
    raw = hatt.hatt(y, z, philox.sketch(9, tt.modes(y), l))
    for k in range(len(raw) - 1):
        q = tt.V(raw[k])
        assert np.allclose(q.T @ q, np.eye(q.shape[1]), atol=1e-12)
    for tol in (1e-2, 1e-5):
        got = rounding.tt_round_left_orth(raw, tol=tol)
        assert tt.rel_err(got, raw) <= tol
    exact = rounding.tt_round_left_orth(raw, tol=1e-13)
    alg1 = rounding.tt_round(raw, tol=1e-13)
    assert tt.ranks(exact) == tt.ranks(alg1)
    assert tt.rel_err(exact, alg1) <= 1e-12


@pytest.mark.parametrize("shape", [(6, 10, 12, 12), (7, 8, 10, 12)])
def test_tolerance_rule_meets_tol_against_explicit_product(shape):
    """The tolerance rule truncates at tol sqrt(3)/2 and accepts only when
    the captured range leaves ||z||^2 - ||X||^2 <= (tol/2)^2 ||z||^2, so the
    result is within tol of z; checked through the difference TT against the
    explicit PKP cores (no cancellation)."""
    d, n, r, s = shape
    y, z = wk.spectral_pair(504 + d, d, n, r, s)
    outs, l, att, ok = adapt.hatt_adaptive([(y, z)], tol=1e-6, seed=3)
    assert ok
    zz = tt.pkp(y, z)
    assert tt.rel_err(outs[0], zz) <= 1e-6
    # the truncation share alone: tol sqrt(3)/2 of ||z|| on the projection
    raw = hatt.hatt(y, z, philox.sketch(3 + att - 1, tt.modes(y), l))
    cap2 = tt.norm(zz) ** 2 - tt.norm(raw) ** 2
    assert cap2 <= max(0.25e-12, 256 * np.finfo(float).eps) * tt.norm(zz) ** 2


def test_hatt2_sketches_equal_explicit_truncated_recursion():
    """eq. HPCRL--2 written out on the explicit PKP train: W^{(d-1)} by the
    definition, then at each bond its SVD truncated to sigma > ep sigma_1 and
    W^{(k-1)} = H(A_k x_3 trunc(W^{(k)})) H(R_k)^T; the oracle's HaTT-2
    (sandwich form, never forming A) keeps the same number of terms and gives
    the same sketches (the truncated product U S V^T has no gauge freedom)."""
    y, z = _rand_pair(9, [4, 5, 4, 5, 4], 3, 3)
    l, R = _setup(y, z, 6)
    ep = 0.3
    w2, used = hatt.hpcrl(y, z, R, variant=2, ep=ep, return_split_ranks=True)
    a = tt.pkp(y, z)
    d = len(a)
    wb = tt.H(a[d - 1]) @ tt.H(R[d - 1]).T
    assert np.allclose(w2[d - 1], wb, rtol=0, atol=1e-13 * np.abs(wb).max())
    for b in range(d - 1, 1, -1):
        u, sg, vt = np.linalg.svd(wb, full_matrices=False)
        keep = max(1, int(np.sum(sg > ep * sg[0])))
        assert used[b] == keep
        assert keep < len(sg)          # really truncated
        wt = (u[:, :keep] * sg[:keep]) @ vt[:keep]
        c = b - 1
        r0, n, _ = a[c].shape
        wb = (tt.V(a[c]) @ wt).reshape(r0, n * wt.shape[1]) @ tt.H(R[c]).T
        assert np.allclose(w2[b - 1], wb, rtol=0, atol=1e-12 * np.abs(wb).max())
