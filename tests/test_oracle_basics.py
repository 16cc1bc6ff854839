"""Pins of the oracle's TT basics, PKP, norms and generator against facts
that do not come from the oracle itself: brute force on full tensors, closed
forms, and published known-answer vectors."""

import math
import os

import numpy as np
import pytest

import workloads as wk
from oracle import flops, philox, plan, tt
from oracle.hatt import _fold, _vec, core_update_row, wl_column

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_tt(rng, n, ranks):
    return [rng.standard_normal((ranks[k], n[k], ranks[k + 1])) for k in range(len(n))]


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_sketch_statistics_and_shape():
    n, ell = [8, 16, 8], [1, 12, 10, 1]
    r = philox.sketch(5, n, ell)
    assert [c.shape for c in r] == [(1, 8, 12), (12, 16, 10), (10, 8, 1)]
    g = philox.gaussian_stream(5, 1, 200000)
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.01
    # variance 1/(l_{k-1} n_k l_k) per Def. 2.1
    assert abs(r[1].var() * 12 * 16 * 10 - 1.0) < 0.15
    # distinct cores and seeds give different streams; same seed repeats
    assert not np.allclose(philox.gaussian_stream(5, 0, 64), philox.gaussian_stream(5, 1, 64))
    assert not np.allclose(philox.gaussian_stream(5, 0, 64), philox.gaussian_stream(6, 0, 64))
    assert np.array_equal(philox.gaussian_stream(5, 2, 33), philox.gaussian_stream(5, 2, 40)[:33])


def test_kronecker_vec_identity_and_folds():
    # eq. (kronecker_product_times_vec): (A kron B) v = vec(B V A^T), V = v|^{s}_{n}
    rng = np.random.default_rng(0)
    m, n, r, s = 3, 4, 5, 2
    A, B = rng.standard_normal((m, n)), rng.standard_normal((r, s))
    v = rng.standard_normal(n * s)
    lhs = np.kron(A, B) @ v
    Vm = v.reshape(n, s).T                      # column-major fold into s x n
    assert np.allclose(lhs, (B @ Vm @ A.T).flatten(order="F"), rtol=0, atol=1e-13)
    assert np.array_equal(_fold(v, n, s), Vm)
    assert np.array_equal(_vec(Vm), v)
    # one W_L column equals the explicit PKP slice times a column of W
    yi, zi = rng.standard_normal((3, 4)), rng.standard_normal((2, 5))   # r0 x r1, s0 x s1
    u = rng.standard_normal(4 * 5)
    assert np.allclose(wl_column(zi, u, yi), np.kron(yi, zi) @ u, atol=1e-13)
    # one row of the core update equals M(g,:) times the explicit PKP slice
    yn, zn = rng.standard_normal((4, 3)), rng.standard_normal((5, 2))   # r1 x r2, s1 x s2
    mrow = rng.standard_normal(4 * 5)
    assert np.allclose(core_update_row(zn, mrow, yn), mrow @ np.kron(yn, zn), atol=1e-13)


def test_full_matches_slice_products():
    rng = np.random.default_rng(1)
    n, rk = [3, 4, 2, 3], [1, 2, 3, 2, 1]
    a = _rand_tt(rng, n, rk)
    f = tt.full(a)
    for _ in range(20):
        idx = tuple(int(rng.integers(0, nk)) for nk in n)
        prod = np.eye(1)
        for k, i in enumerate(idx):
            prod = prod @ a[k][:, i, :]
        assert abs(f[idx] - prod[0, 0]) < 1e-13


def test_pkp_is_elementwise_product_bruteforce():
    y, z = wk.tiny_pair(3)
    a = tt.pkp(y, z)
    assert tt.ranks(a) == [1, 9, 9, 9, 9, 9, 1]
    fy, fz = tt.full(y), tt.full(z)
    assert np.allclose(tt.full(a), fy * fz, rtol=0, atol=1e-14 * np.abs(fy * fz).max())


def test_norms_three_routes():
    y, z = wk.tiny_pair(4)
    a = tt.pkp(y, z)
    ref = np.linalg.norm(tt.full(y) * tt.full(z))
    assert abs(tt.norm(a) - ref) < 1e-13 * ref
    assert abs(math.sqrt(tt.inner_gram(a, a)) - ref) < 1e-12 * ref


def test_rel_err_resolves_tiny_differences():
    rng = np.random.default_rng(5)
    a = _rand_tt(rng, [4, 5, 4], [1, 3, 3, 1])
    b = [c.copy() for c in a]
    b[1] = b[1] + 1e-12 * rng.standard_normal(b[1].shape)
    ref = np.linalg.norm(tt.full(a) - tt.full(b)) / np.linalg.norm(tt.full(b))
    got = tt.rel_err(a, b)
    assert 1e-14 < ref and abs(got - ref) < 1e-3 * ref
    assert tt.rel_err(a, a) < 1e-15


def test_orthogonalizations_keep_tensor_and_orthogonality():
    rng = np.random.default_rng(6)
    a = _rand_tt(rng, [3, 4, 5, 3], [1, 3, 4, 3, 1])
    fa = tt.full(a)
    r = tt.orthogonalize_rl(a)
    l = tt.orthogonalize_lr(a)
    assert np.allclose(tt.full(r), fa, atol=1e-12)
    assert np.allclose(tt.full(l), fa, atol=1e-12)
    for k in range(1, 4):
        h = tt.H(r[k])
        assert np.allclose(h @ h.T, np.eye(h.shape[0]), atol=1e-13)
    for k in range(3):
        v = tt.V(l[k])
        assert np.allclose(v.T @ v, np.eye(v.shape[1]), atol=1e-13)


def test_clamp_rules():
    n = [4] * 6
    assert plan.clamp_ell(n, [1, 3, 3, 3, 3, 3, 1], [1, 3, 3, 3, 3, 3, 1], 9) == [1, 4, 9, 9, 9, 4, 1]
    rng = np.random.default_rng(7)
    for _ in range(50):
        d = int(rng.integers(2, 8))
        n = [int(x) for x in rng.integers(1, 6, size=d)]
        rx = wk.feasible_ranks(n, int(rng.integers(1, 6)))
        ry = wk.feasible_ranks(n, int(rng.integers(1, 6)))
        ell = plan.clamp_ell(n, rx, ry, int(rng.integers(1, 30)))
        assert ell[0] == ell[d] == 1
        for k in range(1, d):
            assert 1 <= ell[k] <= rx[k] * ry[k]
            assert ell[k] <= ell[k - 1] * n[k - 1]
            assert ell[k - 1] <= n[k - 1] * ell[k]


def test_complexity_closed_forms_printed_in_paper():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "complexity_closed_forms.txt")) if l.strip() and l[0] != "#"]
    for row in rows:
        r, s = int(row[0]), int(row[1])
        sp = flops.speedup_models(r, s, r * s)
        assert abs(sp["tt_rounding"] - 13.0 / (6 + 4.0 / s + 4.0 / r)) < 1e-12
        assert abs(sp["randorth"] - 10.0 / (6 + 4.0 / s + 4.0 / r)) < 1e-12
        if r == s:
            sq = flops.speedup_models(r, r, r)
            assert abs(sq["tt_rounding"] - (5 * r * r + 6 * r + 2) / 14.0) < 1e-12
            assert abs(sq["randorth"] - (4 * r + 6) / 14.0) < 1e-12
    # the model ratio of the Table 4.1 rows is the SP(l) of the text
    t = flops.table41(10, 8, 5, 6, 17)
    assert abs(t["tt_rounding"] / t["hatt1"] - flops.speedup_models(5, 6, 17)["tt_rounding"]) < 1e-12
    assert abs(t["randorth"] / t["hatt1"] - flops.speedup_models(5, 6, 17)["randorth"]) < 1e-12


def test_bond_flop_counter_matches_table_for_uniform_interior():
    # with uniform ranks everywhere (boundary ranks forced equal) the per-bond
    # counter reduces to the CHATT leading terms: HPCRL n r s l (2r+2s+2l) and
    # the sweep n r s l (2r+2s+4l) per core, up to the -1/-2 corrections.
    d, n, r, s, l = 6, 5, 4, 3, 7
    nn = [n] * d
    rx, ry, ll = [r] * (d + 1), [s] * (d + 1), [l] * (d + 1)
    got = flops.hatt1_bonds(nn, rx, ry, ll)
    hp = (d - 2) * n * r * s * l * (2 * r + 2 * s + 2 * l)
    assert abs((got["wl"] + got["wr"]) - hp) < 1e-9 * hp
    sweep_leading = (d - 1) * n * r * s * l * (4 * l) + (d - 1) * n * r * s * l * (2 * r + 2 * s)
    assert abs((got["xw"] + got["proj"] + got["update"]) - sweep_leading) < 1e-9 * sweep_leading
