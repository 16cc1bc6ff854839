"""GPU parity of the three-factor recompression x (.) y (.) w (called through
the C ABI) against the oracle's three-factor HaTT: relative Frobenius error
1e-10 through the difference TT, kept ranks and widths exact."""

import sys

import numpy as np
import pytest
import torch

import workloads as wk
from oracle import adapt, hatt3 as ohatt3, philox, plan, rounding, tt
import paper_2410_04385_amd as H

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _triple(seed, n, r, s, t):
    rng = np.random.default_rng(seed)
    return tuple(wk.gaussian_tt(rng, n, wk.feasible_ranks(n, q)) for q in (r, s, t))


def _widths(x, y, w, ell):
    return plan.clamp_ell(tt.modes(x), tt.ranks(x), [a * b for a, b in zip(tt.ranks(y), tt.ranks(w))], ell)


CASES = [
    ([9], 1, 1, 1, 1),                # d = 1
    ([6, 7], 3, 2, 2, 4),             # d = 2: no HPCRL recursion
    ([5, 6, 5], 3, 2, 3, 9),          # d = 3
    ([3, 5, 2, 4, 3], 2, 3, 2, 7),    # uneven modes and ranks
    ([1, 4, 1, 3], 2, 2, 2, 3),       # modes of size 1
    ([2] * 12, 4, 3, 5, 24),          # binary modes (the QTT shape), every M reduced over two slices
    ([17, 33, 9, 5], 5, 6, 4, 30),    # ragged GEMM tiles
    ([8, 6, 7, 6, 8], 7, 6, 8, 70),   # wide frames: panelled QR above 64 columns
]


@pytest.mark.parametrize("n,r,s,t,ell", CASES)
def test_hatt3_explicit_sketch_matches_oracle(n, r, s, t, ell):
    x, y, w = _triple(sum(n) * 5 + ell, n, r, s, t)
    l = _widths(x, y, w, ell)
    R = wk.gaussian_sketch(np.random.default_rng(ell + 1), n, l)
    _say(f"hatt_recompress3 explicit sketch n={n} r,s,t={r},{s},{t} ell={l}")
    res = H.recompress3(H.TT.from_cores([x]), H.TT.from_cores([y]), H.TT.from_cores([w]), ell,
                        sketch=H.TT.from_cores(R))
    torch.cuda.synchronize()
    ref = ohatt3.hatt3(x, y, w, R)
    got = res.train(0)
    assert res.ranks[0].cpu().tolist() == l
    assert tt.rel_err(got, ref) <= TOL
    for c in range(len(n) - 1):
        v = tt.V(got[c])
        assert np.allclose(v.T @ v, np.eye(v.shape[1]), atol=1e-12)


@pytest.mark.parametrize("kw", [{"tol": 1e-3}, {"max_rank": 6}, {"tol": 1e-2, "max_rank": 9}])
def test_hatt3_philox_sketch_truncated_matches_oracle(kw):
    n = [4, 5, 6, 5, 4]
    x, y, w = _triple(77, n, 3, 4, 3)
    l = _widths(x, y, w, 20)
    _say(f"hatt_recompress3 philox sketch n={n} ell={l} {kw}")
    res = H.recompress3(H.TT.from_cores([x]), H.TT.from_cores([y]), H.TT.from_cores([w]), 20, seed=11, **kw)
    torch.cuda.synchronize()
    ref = rounding.tt_round_left_orth(ohatt3.hatt3(x, y, w, philox.sketch(11, n, l)),
                                      max_rank=kw.get("max_rank"), tol=kw.get("tol", 0.0))
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(ref)
    assert tt.rel_err(got, ref) <= TOL


def test_hatt3_trig_cube_adaptive_closed_form_and_oracle_decisions():
    """u of rank 6 on a 32^3 grid: u^3 has TT ranks 6J + 1 = 19 (J = 3); the
    tolerance mode takes the same widths and attempts as the oracle's rule."""
    u = wk.trig_u(4, n=32, terms=6, nfreq=3)
    U = H.TT.from_cores([u])
    _say("hatt_recompress3_adaptive trig cube n=32 J=3 tol=1e-9")
    res, ell, att = H.recompress3_adaptive(U, U, U, 1e-9, seed=1)
    torch.cuda.synchronize()
    outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(u, u, u)], tol=1e-9, seed=1)
    assert ok
    assert ell == l_ref and att == att_ref
    got = res.train(0)
    assert tt.ranks(got) == [1, 19, 19, 1]
    assert tt.rel_err(got, outs[0]) <= TOL
    ref = tt.full(u) ** 3
    assert np.linalg.norm(tt.full(got) - ref) <= 1e-9 * np.linalg.norm(ref)


def test_hatt3_qtt_cube_matches_two_products_and_closed_form():
    """The Allen-Cahn shape (QTT, mode size 2, order 3D): phi^3 in one pass
    agrees with the oracle's three-factor rule and with the closed form at
    sampled grid points."""
    D = 4
    phi, amp, ks = wk.qtt_trig_field(3, D, terms=3)
    P = H.TT.from_cores([phi])
    _say(f"hatt_recompress3_adaptive QTT phi^3 D={D} (order {3 * D})")
    res, ell, att = H.recompress3_adaptive(P, P, P, 1e-8, seed=2)
    torch.cuda.synchronize()
    outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(phi, phi, phi)], tol=1e-8, seed=2)
    assert ok and ell == l_ref and att == att_ref
    got = res.train(0)
    assert tt.ranks(got) == tt.ranks(outs[0])
    assert tt.rel_err(got, outs[0]) <= TOL
    ref = tt.full(phi) ** 3
    assert np.linalg.norm(tt.full(got) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_hatt3_rejects_batches_and_nonfinite():
    n = [3, 4, 3]
    x, y, w = _triple(5, n, 2, 2, 2)
    X = H.TT.from_cores([x, x])
    with pytest.raises(H.HattError):
        H.recompress3(X, X, X, 5)
    bad = [c.copy() for c in w]
    bad[1][0, 0, 0] = np.nan
    _say("hatt_recompress3_adaptive non-finite w")
    with pytest.raises(H.HattError) as e:
        H.recompress3_adaptive(H.TT.from_cores([x]), H.TT.from_cores([y]), H.TT.from_cores([bad]), 1e-6)
    assert e.value.status == -6
    assert "w train 0" in str(e.value)
