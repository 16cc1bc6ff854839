"""The tolerance mode over an uneven batch (hatt_recompress_batched_adaptive,
through the C ABI): every pair takes its own widths, and each equals the
single-pair tolerance mode with seed + p (widths, attempts, kept ranks, and
the values to 1e-13), and the oracle's tolerance rule on that pair (widths
and attempts exactly, values to the parity tolerance 1e-10), with the error
against z = x (.) y within tol."""

import sys

import numpy as np
import pytest
import torch

import workloads as wk
from oracle import adapt, tt
import paper_2410_04385_amd as H

pytestmark = pytest.mark.gpu

TOL = 1e-10

# (d, n, r_x, r_y): spectral pairs small enough for the oracle, whose exact
# ranks r_x r_y (up to 100) lie far above the start widths max(r_x, r_y) + 8,
# so the pairs need different numbers of attempts (1 to 4)
SHAPES = [(6, 8, 4, 6), (7, 12, 8, 5), (5, 16, 10, 10), (8, 4, 6, 6), (6, 10, 3, 9), (4, 6, 2, 2)]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _batch(seed0):
    raw, pairs = [], []
    for p, (d, n, rx, ry) in enumerate(SHAPES):
        y, z = wk.spectral_pair(seed0 + p, d, n, rx, ry)
        raw.append((y, z))
        pairs.append((H.TT.from_cores([y]), H.TT.from_cores([z])))
    return raw, pairs


@pytest.mark.parametrize("tol", [1e-6, 1e-2])
def test_batched_tolerance_mode_matches_single_pair_calls_and_oracle(tol):
    """At 1e-6 every pair grows to its exact rank; at 1e-2 two of them stop
    below it and truncate."""
    raw, pairs = _batch(900)
    seed = 300
    _say(f"hatt_recompress_batched_adaptive: {len(pairs)} uneven pairs, tol {tol}")
    res, ells, atts = H.recompress_batched_adaptive(pairs, tol, seed=seed)
    torch.cuda.synchronize()
    _say(f"  attempts {atts}, widest bond per pair {[max(e) for e in ells]}")
    assert len(set(atts)) > 1 and max(atts) > 1
    for p, ((y, z), (X, Z)) in enumerate(zip(raw, pairs)):
        one, ell1, att1 = H.recompress_adaptive(X, Z, tol, seed=seed + p)
        torch.cuda.synchronize()
        got, single = res[p].train(0), one.train(0)
        assert ells[p] == ell1 and atts[p] == att1
        assert tt.ranks(got) == tt.ranks(single)
        assert tt.rel_err(got, single) <= 1e-13
        outs, l_ref, att_ref, ok = adapt.hatt_adaptive([(y, z)], tol=tol, seed=seed + p)
        assert ok and ells[p] == l_ref and atts[p] == att_ref
        assert tt.ranks(got) == tt.ranks(outs[0])
        assert tt.rel_err(got, outs[0]) <= TOL
        assert tt.rel_err(got, tt.pkp(y, z)) <= tol


def test_batched_tolerance_mode_smallest_workspace_gives_the_same_result():
    """With the minimum workspace a round runs fewer pairs side by side (down
    to one); the launches per pair are the same, so the results are equal bit
    for bit."""
    raw, pairs = _batch(950)
    tol, seed = 1e-6, 40
    plan = H.batched_adaptive_plan(pairs, tol, seed=seed)
    assert plan["ws_min"] < plan["ws_full"]
    _say("hatt_recompress_batched_adaptive: full workspace, then the minimum")
    a, ella, atta = H.recompress_batched_adaptive(pairs, tol, seed=seed)
    small = torch.empty(plan["ws_min"], dtype=torch.uint8, device="cuda")
    b, ellb, attb = H.recompress_batched_adaptive(pairs, tol, seed=seed, workspace=small)
    torch.cuda.synchronize()
    assert ella == ellb and atta == attb
    for ra, rb in zip(a, b):
        ga, gb = ra.train(0), rb.train(0)
        assert tt.ranks(ga) == tt.ranks(gb)
        assert all(np.array_equal(u, v) for u, v in zip(ga, gb))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batched_tolerance_mode_start_widths_and_precision(prec):
    """Start widths per pair (here the accepted widths of a first run, every
    bond at its exact rank) and FP32 range finding: every pair equals the
    single-pair call with the same start widths, seed and precision.  In FP64
    each pair is accepted at once; in FP32 a pair whose captured range misses
    tol / 2 by the FP32 rounding of its sketches (measured 1.6e-6 at tol
    1e-6 before the switch) takes one more attempt in FP64."""
    raw, pairs = _batch(990)
    tol, seed = 1e-6, 77
    _say(f"hatt_recompress_batched_adaptive {prec}: default start, then the accepted widths as start")
    _, ells, _ = H.recompress_batched_adaptive(pairs, tol, seed=seed, precision=prec)
    res, ell2, att2 = H.recompress_batched_adaptive(pairs, tol, seed=seed, ell_init=ells, precision=prec)
    torch.cuda.synchronize()
    _say(f"  attempts from the accepted widths: {att2}")
    assert ell2 == ells
    if prec == "f64":
        assert att2 == [1] * len(pairs)
    else:
        assert all(a in (1, 2) for a in att2) and 2 in att2
    for p, (X, Z) in enumerate(pairs):
        one, ell1, att1 = H.recompress_adaptive(X, Z, tol, seed=seed + p, ell_init=ells[p], precision=prec)
        torch.cuda.synchronize()
        assert ell1 == ell2[p] and att1 == att2[p]
        got, single = res[p].train(0), one.train(0)
        assert tt.ranks(got) == tt.ranks(single)
        assert tt.rel_err(got, single) <= 1e-13
        y, z = raw[p]
        assert tt.rel_err(got, tt.pkp(y, z)) <= tol


def test_batched_tolerance_mode_reports_the_pair_with_nonfinite_input():
    raw, pairs = _batch(1010)
    y, z = raw[2]
    bad = [c.copy() for c in z]
    bad[1][0, 1, 0] = np.inf
    pairs[2] = (pairs[2][0], H.TT.from_cores([bad]))
    _say("hatt_recompress_batched_adaptive: pair 2 holds an infinite entry")
    with pytest.raises(H.HattError) as e:
        H.recompress_batched_adaptive(pairs, 1e-6, seed=1)
    assert e.value.status == -6
    assert "pair 2" in str(e.value) and "y train 0" in str(e.value)
