"""BF16 range finding (HPCRL's sandwich and W_L W_R^T on the BF16 matrix
cores with FP32 accumulation; the sweep and the truncation in FP64) against
the oracle's FP64 HaTT with the same Philox sketch, element by element
through the difference TT.

What BF16 costs: the sketches W^{(k)} carry BF16 rounding (unit roundoff
2^-9 ~ 2e-3) of every operand, so they are perturbed by ~1e-2 relative
after the K-long sums.  A perturbed sketch is still a sketch: the frame
X^{(k)} W^{(k)} is formed and projected in FP64, so the output is an exact
FP64 orthogonal projection of z onto a left-orthonormal frame (checked to
1e-12).  What the perturbation changes is the captured range, where
X^{(k)} has directions outside the product's column space: below exact rank
(the spectral pairs) the result then differs from the FP64 one by a few
times 1e-2, while where X^{(k)} itself has the product's rank (the first
bond of the trig product, any bond at exact widths) the BF16 products add
nothing and what remains is the FP32 storage of the sketches (a few 1e-8,
the same as with FP32 range finding).  The bounds are the measured values
with a margin of four or more."""

import sys

import numpy as np
import pytest
import torch

import workloads as wk
from oracle import hatt as ohatt
from oracle import philox, plan, rounding, tt
import paper_2410_04385_amd as H

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _ell(y, z, ell):
    return plan.clamp_ell(tt.modes(y), tt.ranks(y), tt.ranks(z), ell)


def test_bf16_range_finding_exact_rank():
    """At the exact widths the BF16 sketches still span the whole range of
    each frame; what is left is the FP32 storage of the sketches (measured
    1.7e-8, as with FP32 range finding)."""
    y, z = wk.tiny_pair(11)
    _say("hatt_recompress bf16 tiny exact widths")
    res = H.recompress(H.TT.from_cores([y]), H.TT.from_cores([z]), 9, seed=3, precision="bf16")
    torch.cuda.synchronize()
    err = tt.rel_err(res.train(0), tt.pkp(y, z))
    _say(f"  rel err vs the product {err:.2e}")
    assert err <= 1e-6


def test_bf16_projection_identity_and_closeness_spectral_d8():
    """Spectral pair (d = 8, width 40): the BF16 result is an exact FP64
    orthogonal projection of z (||z||^2 = ||X||^2 + ||z - X||^2 to 1e-12) and
    stays close to the FP64 result with the same sketch, before and after
    truncation to rank 30."""
    y, z = wk.spectral_pair(31, 8, 32, 20, 20)
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    _say("hatt_recompress bf16 vs f64 spectral d=8")
    rb = H.recompress(X, Z, 40, seed=12, precision="bf16")
    r64 = H.recompress(X, Z, 40, seed=12)
    tb = H.recompress(X, Z, 40, max_rank=30, seed=12, precision="bf16")
    t64 = H.recompress(X, Z, 40, max_rank=30, seed=12)
    torch.cuda.synchronize()
    ab, a64 = rb.train(0), r64.train(0)
    zz = tt.pkp(y, z)
    nz, nx = tt.norm(zz), tt.norm(ab)
    resid = tt.rel_err(ab, zz) * nz
    assert abs(nz ** 2 - nx ** 2 - resid ** 2) <= 1e-12 * nz ** 2
    for c in range(len(ab) - 1):
        v = tt.V(ab[c])
        assert np.allclose(v.T @ v, np.eye(v.shape[1]), atol=1e-12)
    d_full = tt.rel_err(ab, a64)
    d_trunc = tt.rel_err(tb.train(0), t64.train(0))
    e_b, e_64 = tt.rel_err(ab, zz), tt.rel_err(a64, zz)
    _say(f"  bf16 vs f64: untruncated {d_full:.2e}, truncated {d_trunc:.2e}; error vs z {e_b:.4f} / {e_64:.4f}")
    assert tt.ranks(tb.train(0)) == tt.ranks(t64.train(0))
    assert d_full <= 0.05 and d_trunc <= 0.05  # measured 7e-3
    assert abs(e_b - e_64) <= 0.01 * e_64


def test_bf16_range_finding_matches_oracle_spectral_order_20():
    """The spectral workload's shape (d = 20, width 40): BF16 range finding
    against the oracle's FP64 HaTT with the same Philox sketch, untruncated
    and truncated to rank 30; each FP32 sketch is kept at unit scale by
    powers of two, so nothing leaves BF16's range along 18 HPCRL steps."""
    cfg = wk.WORKLOADS["spectral"]
    y, z = wk.spectral_pair(1001, cfg["d"], cfg["n"], cfg["r"], cfg["r"])
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    l = _ell(y, z, cfg["ell"])
    raw = ohatt.hatt(y, z, philox.sketch(5, tt.modes(y), l))
    ref = rounding.tt_round_left_orth(raw, max_rank=cfg["max_rank"])
    _say("hatt_recompress bf16 vs oracle spectral d=20")
    a = H.recompress(X, Z, cfg["ell"], seed=5, precision="bf16")
    b = H.recompress(X, Z, cfg["ell"], max_rank=cfg["max_rank"], seed=5, precision="bf16")
    torch.cuda.synchronize()
    zz = tt.pkp(y, z)
    e_raw, e_tr = tt.rel_err(a.train(0), raw), tt.rel_err(b.train(0), ref)
    e_b, e_64 = tt.rel_err(a.train(0), zz), tt.rel_err(raw, zz)
    _say(f"  bf16 vs oracle: untruncated {e_raw:.2e}, rank 30 {e_tr:.2e}; error vs z {e_b:.4f} / {e_64:.4f}")
    assert tt.ranks(b.train(0)) == tt.ranks(ref)
    assert e_raw <= 0.1 and e_tr <= 0.1  # measured 2.4e-2, 2.5e-2
    assert abs(e_b - e_64) <= 0.01 * e_64


def test_bf16_range_finding_accuracy_on_trig_u2():
    """u (.) u on the 256^3 trig grid at width 96 (exact rank 81), tol 1e-8:
    the first bond's frame X^{(1)} W^{(1)} has X^{(1)} of the product's rank
    81, so the BF16 sketch W^{(1)} loses nothing there; the last bond's
    sketch is formed in FP64 and stored in FP32.  Measured 4.0e-8 against the
    oracle and the closed form, the FP32 figure: same ranks, bound 1e-6."""
    cfg = wk.WORKLOADS["trig"]
    u = wk.trig_u(11, n=cfg["n"], terms=2 * cfg["nfreq"], nfreq=cfg["nfreq"])
    U = H.TT.from_cores(u)
    l = _ell(u, u, cfg["ell2"])
    ref = rounding.tt_round_left_orth(ohatt.hatt(u, u, philox.sketch(1, tt.modes(u), l)), tol=cfg["tol"])
    _say("hatt_recompress bf16 trig 256^3 u*u width 96 tol 1e-8")
    got = H.recompress(U, U, cfg["ell2"], tol=cfg["tol"], seed=1, precision="bf16")
    torch.cuda.synchronize()
    g = got.train(0)
    e_or = tt.rel_err(g, ref)
    fu = tt.full(u)
    e_cf = np.linalg.norm(tt.full(g) - fu ** 2) / np.linalg.norm(fu ** 2)
    _say(f"  bf16 ranks {tt.ranks(g)}; vs oracle {e_or:.2e}, vs closed form {e_cf:.2e}")
    assert tt.ranks(g) == tt.ranks(ref) == [1, 81, 81, 1]
    assert e_or <= 1e-6 and e_cf <= 1e-6


def test_bf16_adaptive_runs_and_keeps_projection():
    """Tolerance mode with BF16 range finding (small trig product, tol 1e-3):
    converges, and its result is within the tolerance class of the oracle's
    FP64 tolerance-mode result."""
    from oracle import adapt
    u = wk.trig_u(3, n=24, terms=8, nfreq=4)
    U = H.TT.from_cores(u)
    _say("hatt_recompress_adaptive bf16 small trig tol 1e-3")
    res, ell, att = H.recompress_adaptive(U, U, 1e-3, seed=6, precision="bf16")
    torch.cuda.synchronize()
    outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(u, u)], tol=1e-3, seed=6)
    fu = tt.full(u)
    e = np.linalg.norm(tt.full(res.train(0)) - fu ** 2) / np.linalg.norm(fu ** 2)
    _say(f"  bf16 widths {ell} ({att} attempts) vs oracle {l_ref} ({att_ref}); error vs closed form {e:.2e}")
    assert ok and ell == l_ref and att == att_ref
    assert e <= 1e-3  # measured 5e-9: the tolerance, not the sketch, sets it
    assert tt.rel_err(res.train(0), outs[0]) <= 1e-3


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_low_precision_uneven_batch_against_per_pair_runs(prec):
    """Uneven batch with FP32 / BF16 range finding: every pair equals the
    single-pair call with the same precision and the sketch keyed by seed +
    p (bit for bit: the same launches in the same order on another stream),
    and the FP64 projection identity holds per pair."""
    shapes = [(6, 16, 8, 12), (9, 32, 12, 10), (7, 16, 20, 16), (8, 64, 10, 9)]
    pairs, raw = [], []
    for p, (d, n, rx, ry) in enumerate(shapes):
        y, z = wk.spectral_pair(7000 + p, d, n, rx, ry)
        raw.append((y, z))
        pairs.append((H.TT.from_cores([y]), H.TT.from_cores([z])))
    _say(f"hatt_recompress_batched {prec}: {len(pairs)} uneven pairs")
    res = H.recompress_batched(pairs, 0, max_rank=7, seed=600, precision=prec)
    torch.cuda.synchronize()
    ells = H.batched_plan(pairs, 0, max_rank=7, seed=600, precision=prec)["ell"]
    for p, (X, Z) in enumerate(pairs):
        one = H.recompress(X, Z, ells[p], max_rank=7, seed=600 + p, precision=prec)
        torch.cuda.synchronize()
        a, b = res[p].train(0), one.train(0)
        assert tt.ranks(a) == tt.ranks(b)
        assert tt.rel_err(a, b) <= 1e-13


def test_autotuner_records_uses_and_matches_oracle():
    """Record mode times the candidates of every GEMM and sandwich bucket of
    a spectral recompression (order 8, width 40, rank 30) and keeps the
    fastest; use mode then runs the recorded choices without timing and
    reproduces the recording run bit for bit; both agree with the oracle to
    the parity tolerance (split-K choices change only the summation order)."""
    y, z = wk.spectral_pair(41, 8, 32, 20, 20)
    X, Z = H.TT.from_cores([y]), H.TT.from_cores([z])
    l = _ell(y, z, 40)
    ref = rounding.tt_round_left_orth(ohatt.hatt(y, z, philox.sketch(12, tt.modes(y), l)), max_rank=30)
    H.tune_clear()
    try:
        H.tune("record")
        _say("autotuner: record on a spectral pair d=8")
        a = H.recompress(X, Z, 40, max_rank=30, seed=12)
        torch.cuda.synchronize()
        table = H.tune_table()
        _say("  table:\n" + table)
        assert "gemm" in table and "sandwich" in table
        H.tune("use")
        b = H.recompress(X, Z, 40, max_rank=30, seed=12)
        torch.cuda.synchronize()
        assert H.tune_table() == table
    finally:
        H.tune("off")
        H.tune_clear()
    ga, gb = a.train(0), b.train(0)
    assert tt.ranks(ga) == tt.ranks(gb) == tt.ranks(ref)
    assert all(np.array_equal(p, q) for p, q in zip(ga, gb))
    assert tt.rel_err(ga, ref) <= 1e-10
