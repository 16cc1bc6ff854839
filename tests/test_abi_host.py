"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every declared entry point, planning reproduces the clamp rules, and
bad arguments are rejected before anything is launched."""

import ctypes
import os
import re

import numpy as np
import pytest
import torch

import workloads as wk
from oracle import plan as oplan
from paper_2410_04385_amd import _lib, api
from paper_2410_04385_amd._lib import HattError

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"HATT_API\s+[\w\s\*]+?\b(\w+)\s*\(", src))
    return names


def _cpu_tt(n, ranks, batch=1):
    _, tot = api._offsets(n, ranks)
    return api.TT(torch.zeros(batch * tot, dtype=torch.float64), n, ranks, batch)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared_symbols()
    assert declared == set(_lib.EXPORTED)
    for name in declared:
        assert hasattr(L, name)
    assert "gfx950" in api.version()


def test_plan_matches_oracle_clamps():
    rng = np.random.default_rng(0)
    for _ in range(40):
        d = int(rng.integers(1, 9))
        n = [int(v) for v in rng.integers(1, 7, size=d)]
        rx = wk.feasible_ranks(n, int(rng.integers(1, 7)))
        ry = wk.feasible_ranks(n, int(rng.integers(1, 7)))
        ell = int(rng.integers(1, 40))
        p = api.plan(_cpu_tt(n, rx), _cpu_tt(n, ry), ell)
        assert p["ell"] == oplan.clamp_ell(n, rx, ry, ell)
        _, tot = api._offsets(n, p["ell"])
        assert p["out_elems"] == tot
        assert p["ws_bytes"] > 0


def test_plan_tiny_workload_exact_rank():
    y, z = wk.tiny_pair(0)
    p = api.plan(_cpu_tt([4] * 6, wk.ranks_of(y)), _cpu_tt([4] * 6, wk.ranks_of(z)), 9)
    assert p["ell"] == [1, 4, 9, 9, 9, 4, 1]


def test_per_bond_widths_and_workspace_growth():
    n = [5] * 5
    x = _cpu_tt(n, [1, 4, 4, 4, 4, 1])
    p1 = api.plan(x, x, [1, 3, 5, 7, 2, 1])
    assert p1["ell"] == [1, 3, 5, 7, 2, 1]
    xb = _cpu_tt(n, [1, 4, 4, 4, 4, 1], batch=8)
    p8 = api.plan(xb, xb, [1, 3, 5, 7, 2, 1])
    assert p8["ws_bytes"] > p1["ws_bytes"]


def test_round_plan_capacities_follow_qr_shapes():
    # the PKP of the tiny workload has ranks 9 but boundary modes of size 4
    p = api.round_plan(_cpu_tt([4] * 6, [1, 9, 9, 9, 9, 9, 1]))
    assert p["cap"] == [1, 4, 9, 9, 9, 4, 1]


@pytest.mark.parametrize("bad", ["rank0", "rankd", "modes", "order", "batch"])
def test_shape_errors(bad):
    n = [3, 4, 3]
    x = _cpu_tt(n, [1, 2, 2, 1])
    y = _cpu_tt(n, [1, 2, 2, 1])
    if bad == "rank0":
        y = api.TT(torch.zeros(64, dtype=torch.float64), n, [2, 2, 2, 1])
    elif bad == "rankd":
        y = api.TT(torch.zeros(64, dtype=torch.float64), n, [1, 2, 2, 2])
    elif bad == "modes":
        y = _cpu_tt([3, 5, 3], [1, 2, 2, 1])
    elif bad == "order":
        y = _cpu_tt([3, 4], [1, 2, 1])
    elif bad == "batch":
        y = _cpu_tt(n, [1, 2, 2, 1], batch=2)
    with pytest.raises(HattError) as e:
        api.plan(x, y, 3)
    assert e.value.status == -2


def test_option_errors():
    n = [3, 4, 3]
    x = _cpu_tt(n, [1, 2, 2, 1])
    with pytest.raises(HattError) as e:
        api.plan(x, x, 0)
    assert e.value.status == -1
    with pytest.raises(HattError) as e:
        api.plan(x, x, 3, tol=-1.0)
    assert e.value.status == -1
    with pytest.raises(HattError) as e:
        api.plan(x, x, 3, variant=3)
    assert e.value.status in (-1, -7)


def test_workspace_too_small_is_rejected_before_launch():
    n = [3, 4, 3]
    x = _cpu_tt(n, [1, 2, 2, 1])
    L = _lib.lib()
    xv, k1 = x.view()
    o, k2 = api._opts(3, 0, 0.0, 1, 1, 0.0, 3)
    out = torch.zeros(1000, dtype=torch.float64)
    rk = torch.zeros(8, dtype=torch.int64)
    ws = torch.zeros(16, dtype=torch.uint8)
    st = L.hatt_recompress(ctypes.byref(xv), ctypes.byref(xv), None, ctypes.byref(o),
                           ctypes.c_void_p(out.data_ptr()), 0, ctypes.c_void_p(rk.data_ptr()),
                           ctypes.c_void_p(ws.data_ptr()), 16, None)
    assert st == -3
    assert b"workspace too small" in L.hatt_last_error()


def test_null_arguments_are_rejected():
    L = _lib.lib()
    assert L.hatt_plan(None, None, None, None, None, None) == -1
    assert L.tt_norm_plan(None, None) == -1
    assert L.hatt_sketch_fill(0, 0, None, None, None, None) == -1


def test_unsupported_widths_are_reported():
    # truncating a sketch wider than the library's largest SVD (3072
    # columns) is refused; 1100 columns are truncated
    n = [4096, 4096, 4096]
    x = _cpu_tt(n, [1, 60, 60, 1])
    api.plan(x, x, 1100, tol=1e-6)
    p = api.plan(x, x, 3100)            # no truncation: any width is fine
    assert p["ell"] == [1, 3100, 3100, 1]
    with pytest.raises(HattError) as e:
        api.plan(x, x, 3100, tol=1e-6)
    assert e.value.status == -7
    assert b"SVD" in _lib.lib().hatt_last_error()


def test_perfmodel_matches_oracle_counts():
    from oracle import flops as oflops
    from paper_2410_04385_amd import perfmodel

    n = [6, 7, 5, 8, 6]
    rx, ry, ell = [1, 3, 4, 5, 2, 1], [1, 2, 3, 4, 3, 1], [1, 5, 9, 7, 4, 1]
    a = perfmodel.hatt_round_flops(n, rx, ry, ell, cap=None)
    b = oflops.hatt1_bonds(n, rx, ry, ell)
    assert abs(a["sandwich"] - (b["wl"] + b["update"])) < 1e-6 * a["sandwich"]
    assert abs(a["gemm_f64"] - (b["wr"] + b["xw"] + b["proj"])) < 1e-6 * a["gemm_f64"]
    assert abs(a["qr"] - b["qr"]) < 1e-6 * a["qr"]
    assert perfmodel.chatt_paper(20, 32, 20, 20, 40) == oflops.table41(20, 32, 20, 20, 40)["hatt1"]


def test_qr_method_switch_and_workspace():
    """Method 0 (CholeskyQR2 + fallback) needs more workspace than method 1
    (Householder only); other values are rejected."""
    x = _cpu_tt([32] * 6, [1, 20, 20, 20, 20, 20, 1])
    try:
        api.set_qr_method("householder")
        w1 = api.plan(x, x, 40, max_rank=30)["ws_bytes"]
        api.set_qr_method("cholqr2")
        w0 = api.plan(x, x, 40, max_rank=30)["ws_bytes"]
    finally:
        api.set_qr_method("cholqr2")
    assert w0 > w1
    assert _lib.lib().hatt_set_qr_method(2) == -1
    with pytest.raises(ValueError):
        api.set_qr_method("qr")


def test_batched_plan_matches_per_pair_plans():
    """Uneven batch plan: per-pair widths and output sizes equal the single
    pair plans (seed + p per pair); the width rule max(r, s) + 8; offsets are
    cumulative; the workspace covers one slot per stream."""
    shapes = [([5, 6, 4], [1, 3, 4, 1], [1, 2, 5, 1], 1), ([8] * 6, [1, 6, 7, 8, 7, 6, 1], [1, 5] + [6] * 4 + [1], 2),
              ([4, 4], [1, 3, 1], [1, 3, 1], 1)]
    pairs = [(_cpu_tt(n, rx, b), _cpu_tt(n, ry, b)) for n, rx, ry, b in shapes]
    p = api.batched_plan(pairs, 0, max_rank=5)
    off, roff = p["out_offset"], p["rank_offset"]
    assert off[0] == 0 and roff[0] == 0
    for k, ((x, y), (n, rx, ry, b)) in enumerate(zip(pairs, shapes)):
        req = [1] + [max(rx[j], ry[j]) + 8 for j in range(1, len(n))] + [1]
        single = api.plan(x, y, req, max_rank=5, seed=k)
        assert p["ell"][k] == single["ell"] == oplan.clamp_ell(n, rx, ry, req)
        assert off[k + 1] - off[k] == b * single["out_elems"]
        assert roff[k + 1] - roff[k] == b * (len(n) + 1)
        assert p["ws_bytes"] >= single["ws_bytes"]
    q = api.batched_plan(pairs, 7)
    for k, (n, rx, ry, b) in enumerate(shapes):
        assert q["ell"][k] == oplan.clamp_ell(n, rx, ry, 7)


def test_batched_plan_errors():
    x = _cpu_tt([4, 5], [1, 3, 1])
    y = _cpu_tt([4, 6], [1, 3, 1])
    with pytest.raises(HattError) as e:
        api.batched_plan([(x, x), (x, y)], 4)
    assert e.value.status == -2
    assert b"pair 1" in _lib.lib().hatt_last_error()
    assert _lib.lib().hatt_batched_plan(0, None, None, None, None, None, None, None) == -1


def test_precision_option_validation():
    x = _cpu_tt([4, 5, 6], [1, 3, 4, 1])
    p32 = api.plan(x, x, 6, precision="f32")
    p64 = api.plan(x, x, 6)
    assert p32["ell"] == p64["ell"]
    with pytest.raises(ValueError):
        api.plan(x, x, 6, precision="f16")
    with pytest.raises(HattError) as e:
        api.plan(x, x, 6, precision="f32", variant=2)
    assert e.value.status == -7


def test_fp32_unsupported_ranks_fail_at_plan():
    """The FP32 and BF16 sandwiches run only on the matrix cores (K <= 128
    per product): a factor rank of 130 is refused at plan time; FP64 takes it
    on its vector kernel."""
    x = _cpu_tt([4, 160, 160, 4], [1, 4, 130, 4, 1])
    y = _cpu_tt([4, 160, 160, 4], [1, 4, 4, 4, 1])
    for prec in ("f32", "bf16"):
        with pytest.raises(HattError) as e:
            api.plan(x, y, 90, precision=prec)
        assert e.value.status == -7
    api.plan(x, y, 90)  # FP64 takes it


def _uneven_pairs(seed, count):
    g = np.random.default_rng(seed)
    pairs = []
    for _ in range(count):
        d = int(g.integers(2, 9))
        n = [int(g.choice([2, 4, 8])) for _ in range(d)]
        rx = oplan.clamp_ell(n, [1] * (d + 1), [1] * (d + 1), [1] + [int(g.integers(1, 9))] * (d - 1) + [1])
        ry = oplan.clamp_ell(n, [1] * (d + 1), [1] * (d + 1), [1] + [int(g.integers(1, 9))] * (d - 1) + [1])
        rx = wk.feasible_ranks(n, max(rx))
        ry = wk.feasible_ranks(n, max(ry))
        pairs.append((_cpu_tt(n, rx), _cpu_tt(n, ry)))
    return pairs


def test_rankpred_widths_match_oracle():
    from oracle import rankpred as orp
    pairs = _uneven_pairs(3, 12)
    rows = api.rankpred_rows(pairs)
    g = np.random.default_rng(4)
    pred = np.log(g.uniform(0.5, 80.0, size=(rows, 2))).astype(np.float32)
    for margin, p in ((0.0, 8), (0.15, 8), (0.3, 4)):
        got = api.rankpred_widths(pairs, pred, margin=margin, oversample=p)
        r = 0
        for (x, y), (ell, rho) in zip(pairs, got):
            want_ell, want_rho = orp.widths(pred[r:r + x.d - 1].astype(np.float64), x.n, x.ranks, y.ranks,
                                            margin, p)
            assert ell == want_ell and rho == want_rho
            r += x.d - 1


def test_rankpred_host_errors_and_workspace():
    pairs = _uneven_pairs(5, 3)
    rows = api.rankpred_rows(pairs)
    pred = np.zeros((rows, 2), np.float32)
    with pytest.raises(HattError) as e:
        api.rankpred_widths(pairs, pred, margin=-0.1)
    assert e.value.status == -1
    bad = pred.copy()
    bad[0, 0] = np.nan
    with pytest.raises(HattError) as e:
        api.rankpred_widths(pairs, bad)
    assert e.value.status == -6
    bad[0, 0] = np.inf
    with pytest.raises(HattError) as e:
        api.rankpred_widths(pairs, bad)
    assert e.value.status == -6
    with pytest.raises(ValueError):
        api.rankpred_widths(pairs, pred[:-1])
    x = _cpu_tt([2, 4, 2], [1, 2, 2, 1])
    y = _cpu_tt([2, 4, 4], [1, 2, 2, 1])
    with pytest.raises(HattError) as e:
        api.rankpred_widths([(x, y)], np.zeros((2, 2), np.float32))
    assert e.value.status == -2
    big = _cpu_tt([4096, 4096], [1, 3000, 1])
    with pytest.raises(HattError) as e:
        api.rankpred_widths([(big, big)], np.zeros((1, 2), np.float32))
    assert e.value.status == -7
    L = _lib.lib()
    for b in (1, 63, 64, 65, 1000):
        assert L.hatt_rankpred_ws_bytes(b) == -(-b // 64) * (19586 + 1) * 4
    assert L.hatt_rankpred_ws_bytes(0) == 0


def test_adaptive_start_widths_are_validated():
    x = _cpu_tt([4, 4, 4], [1, 3, 3, 1])
    with pytest.raises(ValueError):
        api.recompress_adaptive(x, x, 1e-6, ell_init=[1, 5, 1])


def test_adaptive_plan_limits_widths_to_the_svd_limit():
    """A QTT pair (order 28, mode size 2) with ranks 60 and 64 has feasible
    widths up to 3840; the tolerance mode plans its workspace for widths clamped to
    the 3072-column truncation, and every width stays feasible."""
    from oracle import plan as oplan
    d = 28
    rx = [1] + [min(2 ** k, 2 ** (d - k), 60) for k in range(1, d)] + [1]
    ry = [1] + [min(2 ** k, 2 ** (d - k), 64) for k in range(1, d)] + [1]
    n = [2] * d
    x, y = _cpu_tt(n, rx), _cpu_tt(n, ry)
    caps = api.adaptive_caps(x, y)
    full = oplan.clamp_ell(n, rx, ry, [1] + [1 << 40] * (d - 1) + [1])
    assert max(full) == 3840
    assert caps == oplan.clamp_ell(n, rx, ry, [min(c, 3072) for c in full])
    assert max(caps) == 3072


def test_plan_rejects_sandwich_shapes_without_a_kernel():
    """Factor ranks 81 on both sides (u2 * u2 on the 256^3 grid) need a
    sandwich no kernel covers: the plan call reports it before any launch."""
    n = [256, 256, 256]
    r = [1, 81, 81, 1]
    with pytest.raises(HattError) as ei:
        api.plan(_cpu_tt(n, r), _cpu_tt(n, r), 96, tol=1e-8)
    assert ei.value.status == -7 and "sandwich" in str(ei.value)
    # u2 * u (ranks 81 and 40) is covered
    p = api.plan(_cpu_tt(n, r), _cpu_tt(n, [1, 40, 40, 1]), 136, tol=1e-8)
    assert p["ell"] == [1, 136, 136, 1]


def test_noalloc_rejects_problems_beyond_its_scratch_before_any_device_call():
    """The static-scratch entry point checks the workspace need on the host:
    the 256^3 trig product needs about 1 GB, beyond the 128 MiB array, and
    is refused with HATT_EWORKSPACE (no GPU is touched, so this runs here)."""
    n = [256, 256, 256]
    u = _cpu_tt(n, [1, 40, 40, 1])
    class _NullStream:
        cuda_stream = 0

    with pytest.raises(HattError) as ei:
        api.recompress_noalloc(u, u, 96, tol=1e-8, out=_cpu_tt(n, [1, 96, 96, 1]),
                               ranks=torch.zeros((1, 4), dtype=torch.int64), stream=_NullStream())
    assert ei.value.status == -3 and "scratch" in str(ei.value)


def test_randorth_plan_matches_oracle_clamps():
    """RandOrth's widths follow the same clamps as HaTT's with the ranks of
    the explicit train (r_k s_k for PKP cores)."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        d = int(rng.integers(2, 7))
        n = [int(v) for v in rng.integers(2, 6, size=d)]
        ra = wk.feasible_ranks(n, int(rng.integers(2, 20)))
        ell = int(rng.integers(1, 30))
        av, keep = _cpu_tt(n, ra).view()
        eo = (ctypes.c_int64 * (d + 1))()
        ws = ctypes.c_size_t(0)
        oe = ctypes.c_int64(0)
        st = _lib.lib().tt_randorth_plan(ctypes.byref(av), ell, None, eo, ctypes.byref(ws), ctypes.byref(oe))
        assert st == 0
        assert list(eo) == oplan.clamp_ell(n, ra, [1] * (d + 1), ell)
        assert ws.value > 0


def test_rankpred_labels_match_oracle():
    """The predictor's targets are computed behind the C ABI: (ln rho_k,
    ln min(cap_k, rho_k + p)) per interior bond, as the oracle defines them;
    ranks below 1 are rejected."""
    from oracle import rankpred as orp
    rng = np.random.default_rng(4)
    for d in (2, 5, 17):
        kept = [1] + rng.integers(1, 300, size=d - 1).tolist() + [1]
        cap = [1] + [k + int(rng.integers(0, 20)) for k in kept[1:-1]] + [1]
        for p in (8, 3):
            got = api.rankpred_labels(kept, cap, oversample=p)
            assert got.dtype == np.float32 and got.shape == (d - 1, 2)
            assert np.allclose(got, orp.labels(kept, cap, p).astype(np.float32))
    with pytest.raises(HattError) as e:
        api.rankpred_labels([1, 0, 1], [1, 4, 1])
    assert e.value.status == -1


def test_per_bond_rank_caps_are_options():
    """max_rank may be given per bond (d+1 entries): the plan takes it; the
    uneven batch, whose pairs differ in order, refuses it."""
    n = [8] * 5
    x = _cpu_tt(n, [1, 4, 6, 6, 4, 1])
    p = api.plan(x, x, 16, max_rank=[0, 3, 0, 9, 2, 0])
    assert p["ell"] == oplan.clamp_ell(n, [1, 4, 6, 6, 4, 1], [1, 4, 6, 6, 4, 1], [1, 16, 16, 16, 16, 1])
    with pytest.raises(ValueError):
        api.plan(x, x, 16, max_rank=[0, 3, 0])
    xv, kx = x.view()
    xs = (_lib.HattTT * 1)(xv)
    caps = _lib.i64_array([0, 3, 0, 9, 2, 0])
    o = _lib.HattOpts(1, 0.0, 16, None, 0, 0.0, 0, 0, caps)
    oo = (ctypes.c_int64 * 2)()
    ro = (ctypes.c_int64 * 2)()
    eo = (ctypes.c_int64 * 6)()
    ws = ctypes.c_size_t(0)
    st = _lib.lib().hatt_batched_plan(1, xs, xs, ctypes.byref(o), oo, ro, eo, ctypes.byref(ws))
    assert st == -1 and "per-bond rank caps" in _lib.lib().hatt_last_error().decode()


def test_plan3_clamps_with_three_factor_ranks_and_rejects_unsupported():
    rng = np.random.default_rng(3)
    for _ in range(20):
        d = int(rng.integers(1, 8))
        n = [int(v) for v in rng.integers(1, 6, size=d)]
        rx, ry, rw = (wk.feasible_ranks(n, int(rng.integers(1, 5))) for _ in range(3))
        ell = int(rng.integers(1, 60))
        p = api.plan3(_cpu_tt(n, rx), _cpu_tt(n, ry), _cpu_tt(n, rw), ell)
        assert p["ell"] == oplan.clamp_ell(n, rx, [a * b for a, b in zip(ry, rw)], ell)
        assert p["ws_bytes"] > 0
    n = [4] * 4
    x = _cpu_tt(n, [1, 3, 3, 3, 1])
    with pytest.raises(HattError) as e:
        api.plan3(x, x, _cpu_tt([4, 4, 4, 3], [1, 3, 3, 3, 1]), 5)
    assert e.value.status == -2
    xb = _cpu_tt(n, [1, 3, 3, 3, 1], batch=2)
    with pytest.raises(HattError) as e:
        api.plan3(xb, xb, xb, 5)
    assert e.value.status == -7
    L = _lib.lib()
    xv, kx = x.view()
    for variant, prec in ((2, 0), (1, 1)):
        o = _lib.HattOpts(variant, 0.1, 5, None, 0, 0.0, 0, prec, None)
        st = L.hatt_plan3(ctypes.byref(xv), ctypes.byref(xv), ctypes.byref(xv), ctypes.byref(o), None, None, None)
        assert st == -7
    assert L.hatt_plan3(ctypes.byref(xv), ctypes.byref(xv), None, ctypes.byref(o), None, None, None) == -1


def test_precision_option_values():
    n = [4] * 5
    x = _cpu_tt(n, [1, 3, 3, 3, 3, 1])
    p64 = api.plan(x, x, 7)
    for prec in ("f32", "bf16"):
        assert api.plan(x, x, 7, precision=prec)["ell"] == p64["ell"]
    with pytest.raises(HattError) as e:
        api.plan(x, x, 7, variant=2, ep=0.1, precision="bf16")
    assert e.value.status == -7
    L = _lib.lib()
    xv, kx = x.view()
    o = _lib.HattOpts(1, 0.0, 7, None, 0, 0.0, 0, 3, None)
    assert L.hatt_plan(ctypes.byref(xv), ctypes.byref(xv), ctypes.byref(o), None, None, None) == -1


def test_tune_mode_and_table_on_the_host():
    api.tune_clear()
    assert api.tune_table() == ""
    for m in ("record", "use", "off"):
        api.tune(m)
    with pytest.raises(ValueError):
        api.tune("fast")
    assert _lib.lib().hatt_tune_mode(3) == -1
    assert _lib.lib().hatt_tune_table(None, 0) == 1


def test_batched_adaptive_plan_matches_single_pair_plans():
    """The batched tolerance mode's plan: per pair, the widths the growth may
    reach are the single-pair plan's, and the output slots are laid out at
    those widths one after the other; the minimum workspace runs any one pair
    and the full one covers the largest pairs side by side."""
    shapes = [(6, 8, 4, 6), (7, 12, 8, 5), (5, 16, 10, 10), (3, 4, 2, 3)]
    pairs = []
    for d, n, rx, ry in shapes:
        nn = [n] * d
        pairs.append((_cpu_tt(nn, wk.feasible_ranks(nn, rx)), _cpu_tt(nn, wk.feasible_ranks(nn, ry))))
    p = api.batched_adaptive_plan(pairs, 1e-6, seed=3)
    off = 0
    for k, (x, y) in enumerate(pairs):
        caps = api.adaptive_caps(x, y)
        assert p["cap"][k] == caps
        assert p["out_offset"][k] == off
        off += api._offsets(x.n, caps)[1] * x.batch
        assert p["rank_offset"][k + 1] - p["rank_offset"][k] == x.batch * (x.d + 1)
    assert p["out_offset"][-1] == off
    assert 0 < p["ws_min"] <= p["ws_full"]
    one = api.batched_adaptive_plan(pairs[2:3], 1e-6, seed=3)
    assert one["ws_min"] <= p["ws_min"] and one["ws_full"] == one["ws_min"]


def test_batched_adaptive_argument_errors():
    nn = [4] * 5
    x = _cpu_tt(nn, wk.feasible_ranks(nn, 3))
    with pytest.raises(ValueError):
        api.batched_adaptive_plan([(x, x), (x, x)], 1e-6, ell_init=[[1, 5, 5, 5, 5, 1]])
    with pytest.raises(ValueError):
        api.batched_adaptive_plan([(x, x)], 1e-6, ell_init=[[1, 5, 1]])
    with pytest.raises(HattError) as e:
        api.batched_adaptive_plan([(x, x)], 0.0)
    assert e.value.status == -1
    y = _cpu_tt([4] * 4, wk.feasible_ranks([4] * 4, 3))
    with pytest.raises(HattError) as e:
        api.batched_adaptive_plan([(x, x), (x, y)], 1e-6)
    assert "pair 1" in str(e.value)
    assert _lib.lib().hatt_batched_adaptive_plan(0, None, None, None, None, None, None, None, None) == -1
