"""GPU parity of the HIP path (called through the C ABI) against the FP64
oracle.  Floating-point results must agree to a relative Frobenius error of
1e-10 (differences taken as a TT, see oracle.tt.rel_err); integer results
(kept ranks, the PKP expansion) must agree exactly."""

import sys

import numpy as np
import pytest
import torch

import workloads as wk
from oracle import hatt as ohatt
from oracle import philox, plan, randorth, rounding, tt
import paper_2410_04385_amd as H

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _pair(seed, n, r, s):
    rng = np.random.default_rng(seed)
    return (wk.gaussian_tt(rng, n, wk.feasible_ranks(n, r)),
            wk.gaussian_tt(rng, n, wk.feasible_ranks(n, s)))


def _ell(y, z, ell):
    return plan.clamp_ell(tt.modes(y), tt.ranks(y), tt.ranks(z), ell)


def _gpu_hatt(ys, zs, ell, **kw):
    x = H.TT.from_cores(ys)
    y = H.TT.from_cores(zs)
    res = H.recompress(x, y, ell, **kw)
    torch.cuda.synchronize()
    return res


def test_sketch_fill_matches_oracle_generator():
    for n, ell, seed in [([4, 5, 6], [1, 3, 7, 1], 1), ([32] * 20, [1] + [40] * 19 + [1], 2 ** 40 + 7)]:
        ell = plan.clamp_ell(n, [1] + [99] * (len(n) - 1) + [1], [1] + [99] * (len(n) - 1) + [1], ell)
        _say(f"sketch_fill n={n[:3]}.. ell={ell[:3]}.. seed={seed}")
        g = H.sketch_fill(seed, n, ell)
        torch.cuda.synchronize()
        ref = philox.sketch(seed, n, ell)
        got = g.to_numpy()
        for a, b in zip(got, ref):
            assert a.shape == b.shape
            assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_hadamard_explicit_is_exact():
    ys, zs = [], []
    for b in range(3):
        y, z = _pair(10 + b, [3, 5, 2, 4], 3, 2)
        ys.append(y)
        zs.append(z)
    _say("tt_hadamard_explicit batch=3 n=[3,5,2,4]")
    out = H.hadamard_explicit(H.TT.from_cores(ys), H.TT.from_cores(zs))
    torch.cuda.synchronize()
    for b in range(3):
        ref = tt.pkp(ys[b], zs[b])
        for a, c in zip(out.to_numpy(b), ref):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("n,r", [([7], 1), ([6, 7], 3), ([4, 5, 4, 3], 3), ([4] * 6, 9), ([3, 8, 5, 2, 6], 5)])
def test_norm_matches_oracle(n, r):
    rng = np.random.default_rng(sum(n) + r)
    trains = [wk.gaussian_tt(rng, n, wk.feasible_ranks(n, r)) for _ in range(2)]
    _say(f"tt_norm n={n} r={r}")
    got = H.norm(H.TT.from_cores(trains)).cpu().numpy()
    for b in range(2):
        ref = np.linalg.norm(tt.full(trains[b]))
        assert abs(got[b] - ref) <= 1e-12 * ref


def test_round_tiny_pkp_rank_cap_and_tol():
    y, z = wk.tiny_pair(5)
    a = tt.pkp(y, z)
    for kw in ({"max_rank": 4}, {"tol": 1e-3}, {"tol": 3e-2, "max_rank": 5}, {}):
        _say(f"tt_round tiny pkp {kw}")
        res = H.round(H.TT.from_cores(a), **kw)
        torch.cuda.synchronize()
        ref = rounding.tt_round(a, max_rank=kw.get("max_rank"), tol=kw.get("tol", 0.0))
        got = res.train(0)
        assert tt.ranks(got) == tt.ranks(ref)
        assert tt.rel_err(got, ref) <= TOL


def test_round_random_ragged_batch():
    n = [5, 7, 3, 6, 4]
    rng = np.random.default_rng(3)
    trains = [wk.spectral_tt(rng, n, wk.feasible_ranks(n, 12)) for _ in range(3)]
    _say("tt_round spectral ragged batch=3 max_rank=6")
    res = H.round(H.TT.from_cores(trains), max_rank=6)
    torch.cuda.synchronize()
    for b in range(3):
        ref = rounding.tt_round(trains[b], max_rank=6)
        got = res.train(b)
        assert tt.ranks(got) == tt.ranks(ref)
        assert tt.rel_err(got, ref) <= TOL


CASES = [
    ([4] * 6, 3, 3, 9),               # tiny workload, exact rank
    ([4] * 6, 3, 3, 4),               # tiny workload, truncated sketch
    ([3, 5, 2, 4, 3], 2, 4, 5),       # r != s, uneven modes
    ([6, 7], 3, 2, 4),                # d = 2
    ([5, 6, 5], 4, 3, 7),             # d = 3
    ([2] * 8, 2, 3, 5),               # binary modes
    ([1, 4, 1, 3], 2, 2, 3),          # modes of size 1
    ([9], 1, 1, 1),                   # d = 1
    ([17, 33, 65, 9], 6, 7, 30),      # ragged tiles in every kernel
    ([5, 6, 7, 6, 5], 19, 17, 23),    # bond ranks 17..20: 4 x 4 x 4 remainder blocks, ragged chunks
    ([4, 8, 8, 8, 4], 20, 18, 40),    # same, r != s on both sandwich sides
    ([7, 9, 8, 7], 7, 7, 44),         # a 44-wide frame: a full third column block in the thin GEMM
    ([6, 9, 7, 5], 7, 6, 35),         # a 35-wide frame: one 4-wide strip in the thin GEMM
]


@pytest.mark.parametrize("n,r,s,ell", CASES)
def test_hatt_explicit_sketch_matches_oracle(n, r, s, ell):
    y, z = _pair(sum(n) * 7 + ell, n, r, s)
    l = _ell(y, z, ell)
    R = wk.gaussian_sketch(np.random.default_rng(ell), n, l)
    _say(f"hatt_recompress explicit sketch n={n} r={r} s={s} ell={l}")
    res = _gpu_hatt(y, z, ell, sketch=H.TT.from_cores(R))
    ref = ohatt.hatt(y, z, R)
    got = res.train(0)
    assert res.ranks[0].cpu().tolist() == l
    assert tt.rel_err(got, ref) <= TOL
    for c in range(len(n) - 1):
        v = tt.V(got[c])
        assert np.allclose(v.T @ v, np.eye(v.shape[1]), atol=1e-12)


# Middle-bond ranks chosen so the sandwich contractions run the
# register-blocked kernel at every K-step count from 1 to 8 (K = bond rank
# padded to 4 on both factors), plus unequal K steps and K beyond 32, which
# take the runtime-K kernel.
SANDWICH_SHAPES = [(4, 3), (8, 7), (12, 10), (16, 14), (24, 21), (28, 26), (32, 30), (22, 26), (36, 33)]


def test_sandwich_wide_free_sides_match_oracle():
    """Bond ranks 56 / 52 beside 16 / 14: the register-blocked sandwich with
    four ZR column blocks and four YL row blocks (every wave in its own block
    column / row) at four K steps."""
    rng = np.random.default_rng(77)
    n = [8, 8, 8, 8, 8]
    y = wk.gaussian_tt(rng, n, [1, 8, 56, 16, 8, 1])
    z = wk.gaussian_tt(rng, n, [1, 8, 52, 14, 8, 1])
    l = _ell(y, z, 30)
    R = wk.gaussian_sketch(np.random.default_rng(78), n, l)
    _say(f"hatt_recompress wide free sides ranks {tt.ranks(y)} / {tt.ranks(z)} ell={l}")
    res = _gpu_hatt([y], [z], 30, sketch=H.TT.from_cores(R))
    assert tt.rel_err(res.train(0), ohatt.hatt(y, z, R)) <= TOL


@pytest.mark.parametrize("r,s", SANDWICH_SHAPES)
def test_sandwich_k_steps_match_oracle(r, s):
    n = [6, 6, 6, 6]
    y, z = _pair(100 * r + s, n, r, s)
    l = _ell(y, z, 13)
    R = wk.gaussian_sketch(np.random.default_rng(r + s), n, l)
    _say(f"hatt_recompress sandwich shapes ranks {tt.ranks(y)} / {tt.ranks(z)} ell={l}")
    res = _gpu_hatt(y, z, 13, sketch=H.TT.from_cores(R))
    assert tt.rel_err(res.train(0), ohatt.hatt(y, z, R)) <= TOL


def test_hatt_exact_rank_reproduces_product():
    y, z = wk.tiny_pair(0)
    _say("hatt_recompress tiny exact rank, seeded")
    res = _gpu_hatt(y, z, 9, seed=99)
    got = res.train(0)
    fz = tt.full(y) * tt.full(z)
    assert np.linalg.norm(tt.full(got) - fz) <= 1e-12 * np.linalg.norm(fz)


def test_hatt_seeded_sketch_matches_oracle_generator():
    y, z = _pair(4, [5, 6, 7, 6, 5], 3, 4)
    l = _ell(y, z, 8)
    seed = 123456789
    _say(f"hatt_recompress seeded n=[5,6,7,6,5] ell={l}")
    res = _gpu_hatt(y, z, 8, seed=seed)
    ref = ohatt.hatt(y, z, philox.sketch(seed, tt.modes(y), l))
    assert tt.rel_err(res.train(0), ref) <= TOL


@pytest.mark.parametrize("kw", [{"max_rank": 4}, {"tol": 1e-2}, {"tol": 0.2, "max_rank": 6}])
def test_hatt_truncated_matches_oracle(kw):
    y, z = _pair(8, [5, 6, 7, 6, 5, 4], 3, 3)
    l = _ell(y, z, 9)
    R = wk.gaussian_sketch(np.random.default_rng(1), tt.modes(y), l)
    _say(f"hatt_recompress truncated {kw}")
    res = _gpu_hatt(y, z, 9, sketch=H.TT.from_cores(R), **kw)
    ref = rounding.tt_round_left_orth(ohatt.hatt(y, z, R), max_rank=kw.get("max_rank"), tol=kw.get("tol", 0.0))
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= TOL


def test_hatt_batched_pairs_match_per_pair_oracle():
    B = 5
    pairs = [_pair(100 + b, [4, 6, 5, 6, 4], 4, 3) for b in range(B)]
    ys = [p[0] for p in pairs]
    zs = [p[1] for p in pairs]
    l = _ell(ys[0], zs[0], 7)
    R = wk.gaussian_sketch(np.random.default_rng(5), tt.modes(ys[0]), l)
    _say("hatt_recompress batch=5 shared sketch max_rank=5")
    res = _gpu_hatt(ys, zs, 7, sketch=H.TT.from_cores(R), max_rank=5)
    for b in range(B):
        ref = rounding.tt_round_left_orth(ohatt.hatt(ys[b], zs[b], R), max_rank=5)
        assert tt.rel_err(res.train(b), ref) <= TOL


def test_hatt_equals_randorth_on_explicit_product_gpu():
    """The GPU path versus RandOrth on the PKP cores (a second oracle route)."""
    y, z = _pair(21, [4, 5, 6, 5], 3, 3)
    l = _ell(y, z, 6)
    R = wk.gaussian_sketch(np.random.default_rng(2), tt.modes(y), l)
    _say("hatt_recompress vs randorth(pkp)")
    res = _gpu_hatt(y, z, 6, sketch=H.TT.from_cores(R))
    assert tt.rel_err(res.train(0), randorth.randorth(tt.pkp(y, z), R)) <= TOL


def test_spectral_workload_full_size():
    """d=20, n=32, r_x=r_y=20, sketch 40, truncation to rank 30, seeded."""
    cfg = wk.WORKLOADS["spectral"]
    y, z = wk.spectral_pair(0, cfg["d"], cfg["n"], cfg["r"], cfg["r"])
    l = _ell(y, z, cfg["ell"])
    seed = 7
    _say("hatt_recompress spectral full size, 1 pair")
    res = _gpu_hatt(y, z, cfg["ell"], seed=seed, max_rank=cfg["max_rank"])
    ref = rounding.tt_round_left_orth(ohatt.hatt(y, z, philox.sketch(seed, tt.modes(y), l)), max_rank=cfg["max_rank"])
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= TOL


def test_round_large_ranks_panel_qr_and_block_jacobi():
    """PKP ranks up to 144: exercises the wide-matrix QR, the panelled
    (block Gram-Schmidt twice + TSQR) QR for more than 128 columns and the
    block Jacobi SVD for more than 139 columns."""
    y, z = _pair(31, [8, 9, 9, 8], 12, 12)
    a = tt.pkp(y, z)
    assert max(tt.ranks(a)) == 144
    for kw in ({"max_rank": 20}, {"tol": 1e-2}):
        _say(f"tt_round pkp ranks {tt.ranks(a)} {kw}")
        res = H.round(H.TT.from_cores(a), **kw)
        torch.cuda.synchronize()
        ref = rounding.tt_round(a, max_rank=kw.get("max_rank"), tol=kw.get("tol", 0.0))
        got = res.train(0)
        assert tt.ranks(got) == tt.ranks(ref)
        assert tt.rel_err(got, ref) <= TOL


def test_hatt_sketch_wider_than_one_panel():
    """Sketch width 150 (> 128 QR columns, > 139 SVD columns), truncated by tol."""
    y, z = _pair(32, [12, 13, 13, 12], 14, 14)
    l = _ell(y, z, 150)
    assert max(l) == 150
    R = wk.gaussian_sketch(np.random.default_rng(3), tt.modes(y), l)
    _say(f"hatt_recompress ell={l} tol=1e-6")
    res = _gpu_hatt(y, z, 150, sketch=H.TT.from_cores(R), tol=1e-6)
    ref = rounding.tt_round_left_orth(ohatt.hatt(y, z, R), tol=1e-6)
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= TOL


@pytest.mark.parametrize("ep", [1e-14, 1e-3, 0.3])
def test_hatt2_matches_oracle(ep):
    """HaTT-2 (truncated SVD split of W^{(k)}, eq. HPCRL--2) against the oracle."""
    y, z = _pair(41, [5, 6, 7, 6, 5], 3, 3)
    l = _ell(y, z, 8)
    R = wk.gaussian_sketch(np.random.default_rng(4), tt.modes(y), l)
    w, used = ohatt.hpcrl(y, z, R, variant=2, ep=ep, return_split_ranks=True)
    for b in range(2, len(y)):   # keep ep away from a singular value of W^{(b)}
        sv = np.linalg.svd(ohatt.hpcrl(y, z, R, variant=1)[b], compute_uv=False)
        assert np.min(np.abs(sv / sv[0] - ep)) > 1e-6
    _say(f"hatt_recompress variant 2 ep={ep} terms={used}")
    res = _gpu_hatt(y, z, 8, sketch=H.TT.from_cores(R), variant=2, ep=ep)
    ref = ohatt.hatt(y, z, R, variant=2, ep=ep)
    assert tt.rel_err(res.train(0), ref) <= TOL


def test_adaptive_matches_oracle_small_trig():
    """Tolerance-driven widths: same growth decisions and result as the oracle."""
    from oracle import adapt
    u = wk.trig_u(3, n=48, terms=12, nfreq=6)
    seed, tol = 17, 1e-8
    _say("hatt_recompress_adaptive small trig u*u tol=1e-8")
    res, ell, att = H.recompress_adaptive(H.TT.from_cores(u), H.TT.from_cores(u), tol, seed=seed)
    torch.cuda.synchronize()
    outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(u, u)], tol=tol, seed=seed)
    assert ok and ell == l_ref and att == att_ref
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(outs[0]) == [1, 25, 25, 1]
    assert tt.rel_err(got, outs[0]) <= TOL


def test_trig_workload_products_at_tolerance():
    """u on the 256^3 grid (40 separable sin/cos terms): u*u and (u*u)*u at
    tol 1e-8 reach the closed-form ranks 81 and 121 and the pointwise values."""
    cfg = wk.WORKLOADS["trig"]
    u = wk.trig_u(11, n=cfg["n"], terms=2 * cfg["nfreq"], nfreq=cfg["nfreq"])
    fu = tt.full(u)
    U = H.TT.from_cores(u)
    _say("hatt_recompress_adaptive trig 256^3 u*u tol=1e-8")
    r2, ell2, att2 = H.recompress_adaptive(U, U, cfg["tol"], seed=1)
    torch.cuda.synchronize()
    u2 = r2.train(0)
    assert tt.ranks(u2) == [1, 81, 81, 1]
    e2 = np.linalg.norm(tt.full(u2) - fu ** 2) / np.linalg.norm(fu ** 2)
    assert e2 <= cfg["tol"]
    _say(f"hatt_recompress_adaptive trig (u*u)*u tol=1e-8 (u*u widths {ell2}, {att2} attempts)")
    r3, ell3, att3 = H.recompress_adaptive(H.TT.from_cores(u2), U, cfg["tol"], seed=2)
    torch.cuda.synchronize()
    u3 = r3.train(0)
    assert tt.ranks(u3) == [1, 121, 121, 1]
    e3 = np.linalg.norm(tt.full(u3) - fu ** 3) / np.linalg.norm(fu ** 3)
    assert e3 <= 3 * cfg["tol"]


def _padded(train, r, seed):
    """The same tensor as ``train`` (d = 3) carried on bonds of rank r: zero
    padding, then a random orthogonal change of basis on each bond."""
    rng = np.random.default_rng(seed)
    c0, c1, c2 = train
    a, b = c1.shape[0], c1.shape[2]
    q1, _ = np.linalg.qr(rng.standard_normal((r, r)))
    q2, _ = np.linalg.qr(rng.standard_normal((r, r)))
    p0 = np.zeros((1, c0.shape[1], r))
    p0[:, :, :a] = c0
    p1 = np.zeros((r, c1.shape[1], r))
    p1[:a, :, :b] = c1
    p2 = np.zeros((r, c2.shape[1], 1))
    p2[:b] = c2
    return [np.einsum("inj,jk->ink", p0, q1), np.einsum("ij,jnk,kl->inl", q1.T, p1, q2),
            np.einsum("ij,jnk->ink", q2.T, p2)]


@pytest.mark.parametrize("r", [100, 145, 200])
def test_round_rank_deficient_wide_bonds(r):
    """TT-Rounding of a rank-30 tensor carried on bonds of rank r: the
    orthogonalisation QRs are rank deficient (and panelled above 128
    columns); the truncation must still find rank 30."""
    base = wk.gaussian_tt(np.random.default_rng(7), [256, 64, 256], [1, 30, 30, 1])
    pad = _padded(base, r, 3)
    _say(f"tt_round rank-deficient padded r={r}")
    res = H.round(H.TT.from_cores([pad]), tol=1e-10)
    torch.cuda.synchronize()
    got = res.train(0)
    ref = rounding.tt_round(pad, tol=1e-10)
    assert tt.ranks(got) == tt.ranks(ref) == [1, 30, 30, 1]
    assert tt.rel_err(got, ref) <= 1e-10


@pytest.mark.parametrize("ell", [60, 128, 150])
def test_hatt_rank_deficient_sketch(ell):
    """u*u for 20 trig terms has exact rank 41 per bond; sketches wider than
    that make every sketched matrix rank deficient: width 60 exercises the
    CholeskyQR2 rejection and Householder fallback, 128 and 150 the
    panelled path."""
    u = wk.trig_u(5, n=256, terms=20, nfreq=10)
    ells = [1, ell, ell, 1]
    _say(f"hatt_recompress rank-deficient sketch ell={ell}")
    U = H.TT.from_cores([u])
    res = H.recompress(U, U, ells, seed=9)
    torch.cuda.synchronize()
    got = res.train(0)
    R = philox.sketch(9, tt.modes(u), ells)
    ref = ohatt.hatt(u, u, R)
    assert tt.rel_err(got, ref) <= 1e-10
    res = H.recompress(U, U, ells, tol=1e-10, seed=9)
    torch.cuda.synchronize()
    got = res.train(0)
    assert tt.ranks(got) == [1, 41, 41, 1]
    assert tt.rel_err(got, rounding.tt_round(ref, tol=1e-10)) <= 1e-9


def test_qr_fallback_mixed_batch():
    """One batch, two pairs of the same shape: a trig product whose sketched
    matrices are rank deficient (width 60 > rank 41, so CholeskyQR2 rejects
    them and Householder TSQR recomputes that pair) and a Gaussian pair of
    full rank (CholeskyQR2 accepted).  Both must match the oracle."""
    u = wk.trig_u(5, n=256, terms=20, nfreq=10)
    g = wk.gaussian_tt(np.random.default_rng(3), [256, 256, 256], [1, 20, 20, 1])
    ells = [1, 60, 60, 1]
    _say("hatt_recompress mixed CholeskyQR2 / fallback batch ell=60")
    X = H.TT.from_cores([u, g])
    Y = H.TT.from_cores([u, g])
    res = H.recompress(X, Y, ells, seed=4)
    torch.cuda.synchronize()
    R = philox.sketch(4, tt.modes(u), ells)
    for b, (y, z) in enumerate([(u, u), (g, g)]):
        assert tt.rel_err(res.train(b), ohatt.hatt(y, z, R)) <= 1e-10


@pytest.mark.parametrize("method", ["householder", "cholqr2"])
def test_qr_methods_agree_with_oracle(method):
    """The spectral pair at reduced order under each QR method."""
    y, z = wk.spectral_pair(21, 8, 32, 20, 20)
    try:
        H.set_qr_method(method)
        _say(f"hatt_recompress spectral d=8 qr={method}")
        res = H.recompress(H.TT.from_cores([y]), H.TT.from_cores([z]), 40, max_rank=30, seed=8)
        torch.cuda.synchronize()
    finally:
        H.set_qr_method("cholqr2")
    R = philox.sketch(8, tt.modes(y), plan.clamp_ell(tt.modes(y), tt.ranks(y), tt.ranks(z), 40))
    ref = rounding.tt_round_left_orth(ohatt.hatt(y, z, R), max_rank=30)
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= 1e-10


def _rule_ell(y, z):
    rx, ry = tt.ranks(y), tt.ranks(z)
    req = [1] + [max(rx[k], ry[k]) + 8 for k in range(1, len(rx) - 1)] + [1]
    return plan.clamp_ell(tt.modes(y), rx, ry, req)


def test_batched_uneven_pairs_match_oracle():
    """Uneven batch of 10 pairs (orders 2..7, modes 3..8, ranks 1..9, some
    pairs with two trains): every train matches the oracle run with the
    pair's own sketch (key seed + p), truncated to rank 6."""
    rng = np.random.default_rng(17)
    pairs, trains = [], []
    for p in range(10):
        d = int(rng.integers(2, 8))
        n = [int(rng.choice([3, 4, 8])) for _ in range(d)]
        rx = wk.feasible_ranks(n, int(rng.integers(1, 10)))
        ry = wk.feasible_ranks(n, int(rng.integers(1, 10)))
        b = 2 if p % 3 == 0 else 1
        ys = [wk.gaussian_tt(rng, n, rx) for _ in range(b)]
        zs = [wk.gaussian_tt(rng, n, ry) for _ in range(b)]
        pairs.append((H.TT.from_cores(ys), H.TT.from_cores(zs)))
        trains.append((ys, zs))
    _say("hatt_recompress_batched: 10 uneven pairs, rule widths, max_rank 6")
    res = H.recompress_batched(pairs, 0, max_rank=6, seed=500)
    torch.cuda.synchronize()
    for p, (ys, zs) in enumerate(trains):
        ell = _rule_ell(ys[0], zs[0])
        R = philox.sketch(500 + p, tt.modes(ys[0]), ell)
        for b in range(len(ys)):
            ref = rounding.tt_round_left_orth(ohatt.hatt(ys[b], zs[b], R), max_rank=6)
            got = res[p].train(b)
            assert tt.ranks(got) == tt.ranks(ref), p
            assert tt.rel_err(got, ref) <= 1e-10, p


def test_batched_workload_sample():
    """The 512-pair uneven workload's distribution (d in 8..32, n in
    {16, 32, 64}, ranks 8..48, spectral cores), first 24 pairs at full size,
    tol 1e-6: the three cheapest pairs and the three of largest r_x r_y
    (panelled frames, the largest SVDs) match the oracle; every pair's kept
    ranks respect the planned capacities."""
    shapes = wk.batched_pair_shapes(3, 24)
    pairs, cores = [], []
    for p, (d, n, rx, ry) in enumerate(shapes):
        y, z = wk.spectral_pair(7000 + p, d, n, rx, ry)
        pairs.append((H.TT.from_cores([y]), H.TT.from_cores([z])))
        cores.append((y, z))
    _say("hatt_recompress_batched: 24 pairs of the uneven workload, tol 1e-6")
    res = H.recompress_batched(pairs, 0, tol=1e-6, seed=900)
    torch.cuda.synchronize()
    cost = [d * n * rx * ry for (d, n, rx, ry) in shapes]
    wide = [rx * ry for (_, _, rx, ry) in shapes]
    for p in sorted(set(np.argsort(cost)[:3].tolist() + np.argsort(wide)[-3:].tolist())):
        y, z = cores[p]
        ell = _rule_ell(y, z)
        ref = rounding.tt_round_left_orth(ohatt.hatt(y, z, philox.sketch(900 + int(p), tt.modes(y), ell)), tol=1e-6)
        got = res[p].train(0)
        assert tt.ranks(got) == tt.ranks(ref)
        assert tt.rel_err(got, ref) <= 1e-9
    for p in range(len(pairs)):
        kept = res[p].ranks[0].cpu().tolist()
        assert all(1 <= k <= c for k, c in zip(kept, res[p].out.ranks))


def test_fp32_range_finding_exact_rank():
    """FP32 range finding at the exact widths (tiny workload): the FP64
    projection onto the FP32-found frame reproduces the product to FP32
    accuracy."""
    y, z = wk.tiny_pair(11)
    _say("hatt_recompress f32 tiny exact widths")
    res = H.recompress(H.TT.from_cores([y]), H.TT.from_cores([z]), 9, seed=3, precision="f32")
    torch.cuda.synchronize()
    err = tt.rel_err(res.train(0), tt.pkp(y, z))
    _say(f"  rel err vs the product {err:.2e}")
    assert err <= 1e-5


def test_fp32_range_finding_projection_identity_and_closeness():
    """Spectral pair (d = 8): with FP32 range finding the output is still an
    exact FP64 orthogonal projection of z onto a left-orthonormal frame, so
    ||z||^2 = ||X||^2 + ||z - X||^2 to FP64 rounding; it stays within FP32
    accuracy of the FP64 result with the same sketch, before and after
    truncation to rank 30."""
    y, z = wk.spectral_pair(31, 8, 32, 20, 20)
    X = H.TT.from_cores([y])
    Z = H.TT.from_cores([z])
    _say("hatt_recompress f32 vs f64 spectral d=8")
    r32 = H.recompress(X, Z, 40, seed=12, precision="f32")
    r64 = H.recompress(X, Z, 40, seed=12)
    t32 = H.recompress(X, Z, 40, max_rank=30, seed=12, precision="f32")
    t64 = H.recompress(X, Z, 40, max_rank=30, seed=12)
    torch.cuda.synchronize()
    a32, a64 = r32.train(0), r64.train(0)
    zz = tt.pkp(y, z)
    nz, nx = tt.norm(zz), tt.norm(a32)
    resid = tt.rel_err(a32, zz) * nz
    assert abs(nz ** 2 - nx ** 2 - resid ** 2) <= 1e-12 * nz ** 2
    d_full = tt.rel_err(a32, a64)
    d_trunc = tt.rel_err(t32.train(0), t64.train(0))
    _say(f"  f32 vs f64: untruncated {d_full:.2e}, truncated {d_trunc:.2e}")
    assert d_full <= 1e-4 and d_trunc <= 1e-4
    assert tt.ranks(t32.train(0)) == tt.ranks(t64.train(0))


def test_fp32_range_finding_full_order():
    """Order 20 (the spectral workload, width 40, no truncation): each FP32
    sketch is kept at unit scale by powers of two, so nothing underflows
    along the 18 HPCRL steps; the result is an FP64 projection of z onto a
    frame found in FP32, and its error ||z - X|| / ||z|| (about 0.5 here: z
    has rank 400 and a slowly decaying spectrum) matches the FP64 run's to
    three digits."""
    cfg = wk.WORKLOADS["spectral"]
    y, z = wk.spectral_pair(1001, cfg["d"], cfg["n"], cfg["r"], cfg["r"])
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    _say("hatt_recompress f32 vs f64 spectral d=20")
    a = H.recompress(X, Z, cfg["ell"], seed=5, precision="f32")
    b = H.recompress(X, Z, cfg["ell"], seed=5)
    torch.cuda.synchronize()
    zz = tt.pkp(y, z)
    e32, e64 = tt.rel_err(a.train(0), zz), tt.rel_err(b.train(0), zz)
    _say(f"  error vs z: f32 {e32:.6f}, f64 {e64:.6f}")
    assert abs(e32 - e64) <= 1e-3 * e64


def test_fp32_range_finding_matches_oracle_spectral_order_20():
    """FP32 range finding (HPCRL on the FP32 matrix cores, the sweep in
    FP64) against the oracle's FP64 HaTT with the same Philox sketch, element
    by element through the difference TT, on the spectral workload's shape
    (d = 20, width 40), untruncated and truncated to rank 30.  The FP32
    sketches differ from the FP64 ones by ~1e-6 relative; the frames found
    with them differ by that times the sketched frame's conditioning, so the
    bound is 1e-3 (the rank-30 truncation itself is ~0.5 away from z)."""
    cfg = wk.WORKLOADS["spectral"]
    y, z = wk.spectral_pair(1001, cfg["d"], cfg["n"], cfg["r"], cfg["r"])
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    l = _ell(y, z, cfg["ell"])
    raw = ohatt.hatt(y, z, philox.sketch(5, tt.modes(y), l))
    ref = rounding.tt_round_left_orth(raw, max_rank=cfg["max_rank"])
    _say("hatt_recompress f32 vs oracle spectral d=20")
    a = H.recompress(X, Z, cfg["ell"], seed=5, precision="f32")
    b = H.recompress(X, Z, cfg["ell"], max_rank=cfg["max_rank"], seed=5, precision="f32")
    torch.cuda.synchronize()
    e_raw, e_tr = tt.rel_err(a.train(0), raw), tt.rel_err(b.train(0), ref)
    _say(f"  f32 vs oracle: untruncated {e_raw:.2e}, rank 30 {e_tr:.2e}")
    assert tt.ranks(b.train(0)) == tt.ranks(ref)
    assert e_raw <= 1e-3 and e_tr <= 1e-3


def test_fp32_range_finding_accuracy_on_trig_u2():
    """u (.) u on the 256^3 trig grid at width 96, tol 1e-8, FP32 range
    finding: u (.) u has exact rank 81 < 96 and the FP64 path reaches it to
    ~1e-13.  With FP32 sketches W^{(k)} the frame X^{(k)} W^{(k)} (formed in
    FP64) picks up X^{(k)} times the sketch's rounding noise, and X^{(k)}
    has directions outside the product's column space, so the captured
    range is off by a few FP32 roundings: same ranks as the oracle, and
    within 1e-6 of both the oracle's FP64 result (same Philox sketch) and
    the closed form (measured ~4e-8): an FP32-class result, not the 1e-8
    configuration."""
    cfg = wk.WORKLOADS["trig"]
    u = wk.trig_u(11, n=cfg["n"], terms=2 * cfg["nfreq"], nfreq=cfg["nfreq"])
    U = H.TT.from_cores(u)
    l = _ell(u, u, cfg["ell2"])
    ref = rounding.tt_round_left_orth(ohatt.hatt(u, u, philox.sketch(1, tt.modes(u), l)), tol=cfg["tol"])
    _say("hatt_recompress f32 trig 256^3 u*u width 96 tol 1e-8")
    got = H.recompress(U, U, cfg["ell2"], tol=cfg["tol"], seed=1, precision="f32")
    torch.cuda.synchronize()
    g = got.train(0)
    assert tt.ranks(g) == tt.ranks(ref) == [1, 81, 81, 1]
    e_or = tt.rel_err(g, ref)
    fu = tt.full(u)
    e_cf = np.linalg.norm(tt.full(g) - fu ** 2) / np.linalg.norm(fu ** 2)
    _say(f"  f32 vs oracle {e_or:.2e}, vs closed form {e_cf:.2e}")
    assert e_or <= 1e-6 and e_cf <= 1e-6


def test_fp32_adaptive_matches_oracle_small_trig():
    """Tolerance mode with FP32 range finding on a small trig product: the
    same widths, attempts and ranks as the oracle's FP64 tolerance mode, and
    the same tensor to FP32 range-finding accuracy (1e-6)."""
    from oracle import adapt
    u = wk.trig_u(3, n=24, terms=8, nfreq=4)
    U = H.TT.from_cores(u)
    _say("hatt_recompress_adaptive f32 small trig tol 1e-8")
    res, ell, att = H.recompress_adaptive(U, U, 1e-8, seed=6, precision="f32")
    torch.cuda.synchronize()
    outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(u, u)], tol=1e-8, seed=6)
    assert ok and ell == l_ref and att == att_ref
    assert tt.ranks(res.train(0)) == tt.ranks(outs[0])
    assert tt.rel_err(res.train(0), outs[0]) <= 1e-6


@pytest.mark.parametrize("ell", [40, 56])
def test_many_pairs_fused_gram_cholesky_wide_frames(ell):
    """34 pairs with sketched frames of 40 and 56 columns: the fused Gram +
    Cholesky kernel with three and four 16-column blocks (pipelined row
    batches; one batch in flight), its register-resident elimination, and the
    rounding's QRs of the same widths, every pair against the oracle."""
    B = 34
    n = [8] * 6
    pairs = [wk.spectral_pair(5000 + b, d=6, n=8, rx=7, ry=8) for b in range(B)]
    ys = [p[0] for p in pairs]
    zs = [p[1] for p in pairs]
    l = _ell(ys[0], zs[0], ell)
    assert max(l) == ell
    R = wk.gaussian_sketch(np.random.default_rng(ell), n, l)
    _say(f"hatt_recompress batch={B} ell={l} max_rank=20 (fused Gram + Cholesky, wide frames)")
    res = _gpu_hatt(ys, zs, ell, sketch=H.TT.from_cores(R), max_rank=20)
    for b in range(B):
        ref = rounding.tt_round_left_orth(ohatt.hatt(ys[b], zs[b], R), max_rank=20)
        got = res.train(b)
        assert tt.ranks(got) == tt.ranks(ref), b
        assert tt.rel_err(got, ref) <= TOL, b


def test_many_pairs_fused_gram_cholesky_long_frames():
    """34 pairs whose frames have up to 640 rows (many row batches per
    fused Gram + Cholesky block): every pair matches the oracle, also the two
    with zero columns in their second factor, whose rank-deficient frames go
    to the Householder fallback."""
    B = 34
    n = [16] * 5
    pairs = [wk.spectral_pair(6000 + b, d=5, n=16, rx=7, ry=8) for b in range(B)]
    for b in (5, 20):
        y, z = pairs[b]
        z = [c.copy() for c in z]
        for c in z[:-1]:
            c[:, :, 1:] = 0.0
        pairs[b] = (y, z)
    ys = [p[0] for p in pairs]
    zs = [p[1] for p in pairs]
    l = _ell(ys[0], zs[0], 40)
    R = wk.gaussian_sketch(np.random.default_rng(40), n, l)
    _say(f"hatt_recompress batch={B} ell={l} max_rank=20 (long frames, two rank-deficient pairs)")
    res = _gpu_hatt(ys, zs, 40, sketch=H.TT.from_cores(R), max_rank=20)
    for b in range(B):
        ref = rounding.tt_round_left_orth(ohatt.hatt(ys[b], zs[b], R), max_rank=20)
        got = res.train(b)
        assert tt.ranks(got) == tt.ranks(ref), b
        assert tt.rel_err(got, ref) <= TOL, b


def test_many_pairs_fused_gram_cholesky():
    """40 pairs in one batch (the CholeskyQR2 Gram matrices are then formed
    inside the factorisation kernel): every pair matches the oracle, also
    the two whose second factor has bond rank 1 in disguise (zero columns), so
    their sketched frames are rank deficient and the Householder fallback
    takes over for those pairs only."""
    B = 40
    n = [8, 8, 8, 8, 8, 8]
    pairs = [wk.spectral_pair(4000 + b, d=6, n=8, rx=6, ry=5) for b in range(B)]
    for b in (3, 17):
        y, z = pairs[b]
        z = [c.copy() for c in z]
        for c in z[:-1]:
            c[:, :, 1:] = 0.0
        pairs[b] = (y, z)
    ys = [p[0] for p in pairs]
    zs = [p[1] for p in pairs]
    l = _ell(ys[0], zs[0], 24)
    R = wk.gaussian_sketch(np.random.default_rng(6), n, l)
    _say("hatt_recompress batch=40 ell=24 max_rank=10 (fused Gram + Cholesky, two rank-deficient pairs)")
    res = _gpu_hatt(ys, zs, 24, sketch=H.TT.from_cores(R), max_rank=10)
    for b in range(B):
        ref = rounding.tt_round_left_orth(ohatt.hatt(ys[b], zs[b], R), max_rank=10)
        got = res.train(b)
        assert tt.ranks(got) == tt.ranks(ref), b
        assert tt.rel_err(got, ref) <= TOL, b


@pytest.mark.parametrize("n,terms,rank", [(48, 12, 25), (64, 20, 41)])
def test_round_explicit_trig_product_wide_r(n, terms, rank):
    """Explicit PKP cores of u (.) u (ranks terms^2: 144, or 400 = four
    Gram-Schmidt panels) rounded at tol 1e-8: the frames hold exactly
    duplicated columns (the (a, b) and (b, a) products), and the first
    left-to-right QR leaves a wide R, whose SVD goes through the QR of R^T.
    Ranks and tensor against the oracle's TT-Rounding of its own PKP cores,
    and the norm of the PKP train against the full tensor."""
    u = wk.trig_u(7, n=n, terms=terms, nfreq=terms // 2)
    U = H.TT.from_cores(u)
    _say(f"tt_hadamard_explicit + tt_norm + tt_round trig {n}^3, {terms} terms")
    A = H.hadamard_explicit(U, U)
    full = tt.full(u) ** 2
    assert abs(float(H.norm(A)[0].item()) - np.linalg.norm(full)) <= 1e-12 * np.linalg.norm(full)
    res = H.round(A, tol=1e-8)
    torch.cuda.synchronize()
    ref = rounding.tt_round(tt.pkp(u, u), tol=1e-8)
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref) == [1, rank, rank, 1]
    assert tt.rel_err(got, ref) <= TOL


@pytest.mark.parametrize("mode", ["dup", "zero"])
def test_norm_and_round_exactly_dependent_wide_frames(mode):
    """Bond rank 400 (four Gram-Schmidt panels of 128 columns) with 150 left
    slices of the middle core duplicated or zero: the right-to-left frames
    have exactly dependent columns.  The norm (right-to-left sweep alone) and
    a TT-Rounding at tol 1e-6 against the oracle's."""
    g = np.random.default_rng(2)
    n, r = 64, 400
    c0 = g.standard_normal((1, n, r))
    c1 = g.standard_normal((r, n, r)) / np.sqrt(r)
    c2 = g.standard_normal((r, n, 1))
    for k in range(150):
        c1[2 * k + 1] = c1[2 * k] if mode == "dup" else 0.0
    cores = [c0, c1, c2]
    A = H.TT.from_cores(cores)
    _say(f"tt_norm / tt_round rank 400 with {mode} slices")
    nrm = float(H.norm(A)[0].item())
    ex = np.linalg.norm(tt.full(cores))
    assert abs(nrm - ex) <= 1e-12 * ex
    res = H.round(A, tol=1e-6)
    torch.cuda.synchronize()
    ref = rounding.tt_round(cores, tol=1e-6)
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= TOL


@pytest.mark.parametrize("shape", [(6, 4, 3, 3, 9), (8, 8, 6, 5, 20), (3, 48, 12, 12, 40)])
def test_randorth_explicit_matches_oracle_and_hatt(shape):
    """GPU RandOrth (Alg. 2) on the GPU's PKP cores against the oracle's
    RandOrth of its own PKP cores with the same explicit sketch, and against
    GPU HaTT with the same seeded sketch (HaTT reorganises exactly these
    products, so the tensors agree)."""
    d, n, r, s, ell = shape
    if d == 3:
        y = wk.trig_u(3, n=n, terms=r, nfreq=r // 2)
        z = wk.trig_u(4, n=n, terms=s, nfreq=s // 2)
    else:
        y, z = wk.spectral_pair(31 + d, d, n, r, s)
    X, Y = H.TT.from_cores(y), H.TT.from_cores(z)
    A = H.hadamard_explicit(X, Y)
    ell_c = plan.clamp_ell(tt.modes(y), tt.ranks(y), tt.ranks(z), ell)
    R = wk.gaussian_sketch(np.random.default_rng(9), tt.modes(y), ell_c)
    _say(f"tt_randorth d={d} n={n} r={r} s={s} ell={ell}")
    got = H.randorth(A, ell, sketch=H.TT.from_cores(R))
    torch.cuda.synchronize()
    ref = randorth.randorth(tt.pkp(y, z), R)
    assert got.ranks[0].tolist() == ell_c
    assert tt.rel_err(got.train(0), ref) <= TOL
    # seeded: the same Philox sketch as hatt_recompress draws
    g2 = H.randorth(A, ell, seed=77, tol=1e-10)
    h2 = H.recompress(X, Y, ell, seed=77, tol=1e-10)
    torch.cuda.synchronize()
    assert g2.ranks[0].tolist() == h2.ranks[0].tolist()
    assert tt.rel_err(g2.train(0), h2.train(0)) <= TOL


def _gpu_power(Y, ell, iters, seed):
    """Power iteration on the GPU (Sec. 5, Example 3): HaTT with the Philox
    sketch keyed by seed + t, the norm, and the normalisation by tt_scale."""
    X = H.TT.from_cores([np.ones((1, k, 1)) for k in Y.n])
    H.scale(X, H.norm(X), invert=True)
    lams = []
    for t in range(iters):
        Z = H.recompress(X, Y, ell, seed=seed + t).out
        nz = H.norm(Z)
        lams.append(nz)
        H.scale(Z, nz, invert=True)
        X = Z
    torch.cuda.synchronize()
    return [float(v.item()) for v in lams], X


@pytest.mark.parametrize("fn", ["qing", "alpine"])
def test_power_iteration_matches_oracle(fn):
    """Twelve power-iteration steps at the paper's width l = 5 on a d = 8
    Qing / Alpine tensor (10 points per mode, rank 8): the estimate sequence
    and the final iterate against the oracle's with the same sketches."""
    from oracle import power
    vals = (wk.qing_values if fn == "qing" else wk.alpine_values)(8)
    y = wk.separable_sum_tt(vals)
    _say(f"power iteration {fn} d=8 l=5, 12 steps")
    lam, X = _gpu_power(H.TT.from_cores(y), 5, 12, 40)
    lam_ref, x_ref = power.power_iteration(y, 5, 12, 40)
    assert np.allclose(lam, lam_ref, rtol=1e-10, atol=0)
    assert tt.rel_err(X.to_numpy(0), x_ref) <= 1e-9


def test_qtt_trig_product_adaptive_matches_oracle():
    """QTT shape of the Allen-Cahn solutions (mode size 2, order 12): phi (.)
    phi at tol 1e-8 by the tolerance mode, same widths, attempts, ranks and
    tensor as the oracle's, and pointwise within tol of the closed form."""
    from oracle import adapt
    phi, a, ks = wk.qtt_trig_field(5, 4, terms=4)
    _say("hatt_recompress_adaptive QTT 16^3 (d=12, n=2) phi*phi tol=1e-8")
    P = H.TT.from_cores(phi)
    res, ell, att = H.recompress_adaptive(P, P, 1e-8, seed=8)
    torch.cuda.synchronize()
    outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(phi, phi)], tol=1e-8, seed=8)
    assert ok and ell == l_ref and att == att_ref
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(outs[0])
    assert tt.rel_err(got, outs[0]) <= TOL
    f = tt.full(phi).reshape(-1) ** 2
    assert np.linalg.norm(tt.full(got).reshape(-1) - f) <= 1e-8 * np.linalg.norm(f)


def test_qtt_allen_cahn_cubic_order_21():
    """phi^3 = (phi (.) phi) (.) phi on the 128^3 grid in QTT format (order
    21, phi of rank 30): both products by the tolerance mode at 1e-8,
    against the closed-form field on all 2^21 points."""
    phi, a, ks = wk.qtt_trig_field(9, 7, terms=15)
    P = H.TT.from_cores(phi)
    _say("QTT order 21: phi*phi, then *phi, tol 1e-8")
    r2, ell2, att2 = H.recompress_adaptive(P, P, 1e-8, seed=1)
    torch.cuda.synchronize()
    u2 = H.TT.from_device_cores(H.kept_cores(r2))
    r3, ell3, att3 = H.recompress_adaptive(u2, P, 1e-8, seed=2)
    torch.cuda.synchronize()
    f = tt.full(phi).reshape(-1)
    g2 = tt.full(r2.train(0)).reshape(-1)
    g3 = tt.full(r3.train(0)).reshape(-1)
    assert np.linalg.norm(g2 - f ** 2) <= 1e-8 * np.linalg.norm(f ** 2)
    assert np.linalg.norm(g3 - f ** 3) <= 3e-8 * np.linalg.norm(f ** 3)
    assert max(r3.ranks[0].tolist()) <= 2 * max(ell3)


# Widths of the third tolerance-mode attempt for (phi (.) phi) (.) phi on the
# 512^3 grid (order 27): bond 13 is 262 wide against an exact rank of 166,
# so the sketched frame there is square (262 x 262) and rank deficient, and
# its QR runs as panels whose later columns add nothing to the earlier ones.
_QTT9_WIDTHS = [1, 2, 4, 8, 16, 32, 64, 65, 65, 43, 38, 76, 131, 262, 149, 124, 86, 65, 43, 38, 38, 38, 32, 16,
                8, 4, 2, 1]


@pytest.mark.parametrize("method", ["cholqr2", "householder"])
def test_hatt_panelled_rank_deficient_square_frames(method):
    """HaTT of a QTT pair whose wide bond needs a panelled QR of a square,
    rank-deficient frame: the untruncated result equals the oracle's
    (same sketch), and its TT-Rounding keeps the oracle's ranks."""
    from oracle import adapt
    phi, _, _ = wk.qtt_trig_field(9, 9, terms=15)
    outs, _, _, ok = adapt.hatt_adaptive([(phi, phi)], tol=1e-8, seed=1)
    assert ok
    u2 = outs[0]
    n = tt.modes(u2)
    l = list(_QTT9_WIDTHS)
    raw = ohatt.hatt(u2, phi, philox.sketch(4, n, l), 1, 0.0)
    ref = rounding.tt_round_left_orth(raw, tol=1e-8)
    X, P = H.TT.from_cores(u2), H.TT.from_cores(phi)
    _say(f"HaTT QTT order 27 widths up to 262, QR method {method}")
    H.set_qr_method(method)
    try:
        got = H.recompress(X, P, l, seed=4)
        rnd = H.recompress(X, P, l, tol=1e-8, seed=4)
        torch.cuda.synchronize()
    finally:
        H.set_qr_method("cholqr2")
    assert tt.ranks(got.train(0)) == tt.ranks(raw)
    assert tt.rel_err(got.train(0), raw) <= TOL
    assert tt.ranks(rnd.train(0)) == tt.ranks(ref)
    assert tt.rel_err(rnd.train(0), ref) <= TOL


def test_adaptive_widths_below_svd_limit():
    """(phi (.) phi) (.) phi on the 512^3 grid (order 27) has feasible widths
    up to 2640 (88 x 30) at the middle bonds, all below the 3072-column
    truncation limit: the tolerance mode plans for them, and its attempts,
    widths, ranks and tensor equal the oracle's."""
    from oracle import adapt
    phi, _, _ = wk.qtt_trig_field(9, 9, terms=15)
    outs, _, _, ok = adapt.hatt_adaptive([(phi, phi)], tol=1e-8, seed=1)
    assert ok
    u2 = outs[0]
    X, P = H.TT.from_cores(u2), H.TT.from_cores(phi)
    caps = H.adaptive_caps(X, P)
    assert max(caps) == 2640
    _say("adaptive plan with feasible widths up to 2640 (QTT order 27)")
    r3, ell3, att3 = H.recompress_adaptive(X, P, 1e-8, seed=2)
    torch.cuda.synchronize()
    ref, l_ref, att_ref, ok = adapt.hatt_adaptive([(u2, phi)], tol=1e-8, seed=2)
    assert ok and ell3 == l_ref and att3 == att_ref
    assert tt.ranks(r3.train(0)) == tt.ranks(ref[0])
    assert tt.rel_err(r3.train(0), ref[0]) <= TOL


def test_per_bond_max_rank_matches_oracle():
    """Per-bond truncation caps (entries <= 0 leave a bond to tol alone):
    spectral pair of order 8, width 40, caps on some bonds plus tol 1e-3,
    against the oracle's TT-Rounding with the same caps."""
    y, z = wk.spectral_pair(77, 8, 16, 12, 10)
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    caps = [0, 5, 0, 17, 3, 0, 11, 0, 0]
    l = _ell(y, z, 40)
    raw = ohatt.hatt(y, z, philox.sketch(21, tt.modes(y), l))
    ref = rounding.tt_round_left_orth(raw, max_rank=[c if c > 0 else None for c in caps], tol=1e-3)
    _say("hatt_recompress per-bond max_rank, spectral d=8")
    got = H.recompress(X, Z, 40, max_rank=caps, tol=1e-3, seed=21)
    torch.cuda.synchronize()
    g = got.train(0)
    assert tt.ranks(g) == tt.ranks(ref)
    assert all(tt.ranks(g)[k] <= caps[k] for k in range(1, 8) if caps[k] > 0)
    assert tt.rel_err(g, ref) <= TOL


def test_check_finite_and_adaptive_rejects_non_finite():
    """tt_check_finite flags exactly the trains with a NaN or an infinity;
    the tolerance mode refuses such inputs with HATT_ENONFINITE."""
    u = [wk.trig_u(s, n=16, terms=4, nfreq=2) for s in (1, 2, 3)]
    bad1 = [c.copy() for c in u[1]]
    bad1[1][0, 3, 1] = np.nan
    bad2 = [c.copy() for c in u[2]]
    bad2[2][2, 0, 0] = np.inf
    A = H.TT.from_cores([u[0], bad1, bad2])
    flags = H.check_finite(A)
    torch.cuda.synchronize()
    assert flags.cpu().tolist() == [1, 0, 0]
    B = H.TT.from_cores(bad1)
    G = H.TT.from_cores(u[0])
    with pytest.raises(H.HattError) as e:
        H.recompress_adaptive(G, B, 1e-8, seed=1)
    assert e.value.status == -6 and "y train 0" in str(e.value)


@pytest.mark.parametrize("shape", [(70, 50, 37), (81, 40, 29), (96, 8, 131)])
def test_sandwich_large_ranks_slice_major_matches_oracle(shape):
    """Factor ranks of 70 to 96 (the u^2 (.) u shape of the trig workload and
    neighbours): the W_L build and the core update take the slice-major
    sandwich (one mode index per block, sketch columns streamed one at a
    time, or six at a time with a ragged last chunk for the rank-8 partner);
    HaTT against the oracle with the same sketch, untruncated."""
    r, s, ell = shape
    rng = np.random.default_rng(r * 1000 + s)
    n = [150, 5, 150]
    y = [rng.standard_normal((1, 150, r)), rng.standard_normal((r, 5, r)) / r, rng.standard_normal((r, 150, 1))]
    z = [rng.standard_normal((1, 150, s)), rng.standard_normal((s, 5, s)) / s, rng.standard_normal((s, 150, 1))]
    l = _ell(y, z, ell)
    assert l == [1, ell, ell, 1]
    ref = ohatt.hatt(y, z, philox.sketch(40 + r, n, l))
    _say(f"hatt_recompress slice-major sandwich r={r} s={s} ell={l}")
    got = _gpu_hatt([y], [z], ell, seed=40 + r)
    assert tt.ranks(got.train(0)) == tt.ranks(ref)
    assert tt.rel_err(got.train(0), ref) <= TOL


@pytest.mark.parametrize("kind", ["gaussian_cap_1100", "spectral_tol"])
def test_round_svd_above_1024_columns(kind):
    """A bond of rank 1296 (n = 36, order 4): the truncation's SVD of a
    1296-column R runs the block Jacobi over global memory (7-column blocks,
    185 rounds per sweep) past the former 1024-column limit; capped at 1100
    (random cores, all singular values of order one) and by tol 1e-8
    (spectral cores), against the oracle's TT-Rounding."""
    n = [36] * 4
    ranks = [1, 36, 1296, 36, 1]
    rng = np.random.default_rng(1296)
    if kind == "gaussian_cap_1100":
        a = wk.gaussian_tt(rng, n, ranks)
        kw = {"max_rank": 1100}
    else:
        a = wk.spectral_tt(rng, n, ranks)
        kw = {"tol": 1e-8}
    _say(f"tt_round {kind}: bond rank 1296 -> SVD of 1296 columns")
    res = H.round(H.TT.from_cores([a]), **kw)
    torch.cuda.synchronize()
    ref = rounding.tt_round(a, max_rank=kw.get("max_rank"), tol=kw.get("tol", 0.0))
    got = res.train(0)
    _say(f"  ranks {tt.ranks(got)} vs {tt.ranks(ref)}")
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= TOL


@pytest.mark.parametrize("n,r,s,batch", [([7], 1, 1, 2), ([4, 5, 6, 3], 3, 4, 3), ([2] * 9, 3, 2, 1),
                                         ([1, 6, 1, 5], 2, 3, 2), ([9, 17, 8], 20, 24, 1)])
def test_hadamard_norm2_matches_explicit(n, r, s, batch):
    """||x (.) y||^2 by the PKP-free Gram recursion against the norm of the
    oracle's explicit PKP train, per train of a batch."""
    xs, ys = [], []
    for b in range(batch):
        x, y = _pair(sum(n) * 3 + r + b, n, r, s)
        xs.append(x)
        ys.append(y)
    _say(f"hatt_hadamard_norm2 n={n} r={r} s={s} batch={batch}")
    got = H.hadamard_norm2(H.TT.from_cores(xs), H.TT.from_cores(ys)).cpu().numpy()
    for b in range(batch):
        ref = tt.norm(tt.pkp(xs[b], ys[b])) ** 2
        assert abs(got[b] - ref) <= 1e-12 * ref


def test_tolerance_mode_meets_tol_on_a_wide_uneven_pair():
    """A pair of the uneven distribution (d 13, n 16, ranks 17 x 42, product
    rank 714) on which the slack test alone accepted a result 4.8e-6 away
    from z at tol 1e-6: with the capture test the result is within tol,
    checked through the difference TT against the explicit product on the
    GPU."""
    shapes = wk.batched_pair_shapes(1, 512)
    d, n, rx, ry = shapes[398]
    assert (d, n, rx, ry) == (13, 16, 17, 42)
    y, z = wk.spectral_pair(20000 + 398, d, n, rx, ry)
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    _say("hatt_recompress_adaptive tol 1e-6 on uneven pair 398 (13, 16, 17 x 42)")
    res, ell, att = H.recompress_adaptive(X, Z, 1e-6, seed=77 + 398, max_attempts=12)
    torch.cuda.synchronize()
    zt = H.hadamard_explicit(X, Z)
    err = H.rel_err(H.kept_cores(res), [zt.core(k, 0) for k in range(d)])
    _say(f"  {att} attempts, max width {max(ell)}, error vs z {err:.2e}")
    assert err <= 1e-6
