"""Host-side pieces of bench.py: the roofline grouping of launch sites by
compiled kernel and its algorithmic flop counts (no GPU)."""

import importlib.util
import os

import pytest

from paper_2410_04385_amd import perfmodel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


REPORT = """\
     100.000 ms       20 calls  sandwich: sandwich update n=32 G=40 RA=20 RI=20 SI=20 SO=20 [sandwich_reg_kernel<24, 2, false>]
      50.000 ms       10 calls  gemm_f64: gemm 400x40x1280 ks=2 [gemm_f64_kernel<64, 32>]
      60.000 ms       10 calls  qr: gemm 1280x40x40 ks=1 flagged [gemm_f64_kernel<64, 32>]
       5.000 ms       10 calls  gemm_f64: splitk_reduce 400x40 ks=2
       9.000 ms       10 calls  qr: chol 40
"""


def test_roofline_groups_sites_by_compiled_kernel():
    b = _bench()
    roof = b._roofline(REPORT, 128, 10, perfmodel)
    # gemm_f64_kernel<64, 32>: 110 ms over 20 launches beats the sandwich's 100 ms
    assert roof["kernel"] == "gemm_f64_kernel<64, 32>"
    assert roof["avg_launch_us"] == pytest.approx(110.0 / 20 * 1000)
    flops = (2 * 400 * 40 * 1280 * 10 + 2 * 1280 * 40 * 40 * 10) * 128
    nbytes = 8 * ((400 * 1280 + 1280 * 40 + 400 * 40) * 10 + (1280 * 40 + 40 * 40 + 1280 * 40) * 10) * 128
    assert roof["algorithmic_flop_per_launch"] == pytest.approx(flops / 20)
    assert roof["algorithmic_TFLOPs"] == pytest.approx(flops / 0.110 / 1e12)
    # 8.2 flop/B is below the FP64 ridge (78.6 TFLOP/s / 8 TB/s = 9.8): HBM-bound
    assert roof["algorithmic_intensity_flop_per_byte"] == pytest.approx(flops / nbytes)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["achieved"] == pytest.approx(nbytes / 0.110 / 1e9)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0)
    # the runner-up kernels, by time: the VALU sandwich (10 ms per step)
    nxt = roof["next_kernels"]
    assert [k["kernel"] for k in nxt] == ["sandwich_reg_kernel<24, 2, false>"]
    assert nxt[0]["ms_per_step"] == pytest.approx(10.0)
    sw_flops = 2.0 * 32 * 40 * (20 * 20 * 20 + 20 * 20 * 20) * 128 * 20
    assert nxt[0]["unit"] == "TFLOP/s" and nxt[0]["achieved"] == pytest.approx(sw_flops / 0.100 / 1e12)


def test_roofline_above_the_ridge_is_matrix_core_bound():
    b = _bench()
    rep = "      10.000 ms        5 calls  gemm_f64: gemm 1024x1024x1024 ks=1 [gemm_f64_kernel<64, 64, 0>]\n"
    roof = b._roofline(rep, 4, 5, perfmodel)
    flops = 2.0 * 1024 ** 3 * 4
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s" and roof["peak"] == 78.6
    assert roof["achieved"] == pytest.approx(flops / 0.002 / 1e12)


def test_sandwich_site_flops():
    b = _bench()
    kern, bound, f, nb = b._site_group(
        "sandwich W_L n=32 G=40 RA=20 RI=20 SI=20 SO=20 [sandwich_reg_kernel<24, 2, true>]", 2)
    assert kern == "sandwich_reg_kernel<24, 2, true>" and bound == "alu"
    # per (i, g): T = C ZR (RI x SI x SO) then YL T (RA x RI x SO), 2 flops per multiply-add
    assert f == 2.0 * 32 * 40 * (20 * 20 * 20 + 20 * 20 * 20) * 2
    # W^{(k)} (r s x l), the n slices of both cores, W_L (r s x n l), once each
    assert nb == 8.0 * (20 * 20 * 40 + 32 * 400 + 32 * 400 + 400 * 32 * 40) * 2
    kern, bound, f, nb = b._site_group("gemm 1280x40x400 ks=1 [gemm_f64_kernel<64, 32>]", 3)
    assert (f, nb) == (2.0 * 1280 * 40 * 400 * 3, 8.0 * (1280 * 400 + 400 * 40 + 1280 * 40) * 3)
    assert b._site_group("qr: chol 40", 1) is None


def test_traffic_record_is_tied_to_batch_precision_and_source():
    """Counter bytes are reported only for the batch and precision they were
    taken at and while the kernel's source is unchanged."""
    import hashlib
    import json

    b = _bench()
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for kernel, ent in data.items():
        with open(os.path.join(ROOT, ent["source"]), "rb") as fh:
            same = hashlib.sha256(fh.read()).hexdigest() == ent["source_sha256"]
        prec = ent["precision"]
        other = "f32" if prec == "f64" else "f64"
        assert b._traffic(kernel, ent["batch"], prec) == (ent["hbm_bytes_per_launch"] if same else None)
        assert b._traffic(kernel, ent["batch"] + 1, prec) is None
        assert b._traffic(kernel, ent["batch"], other) is None
    assert b._traffic("no_such_kernel", 512, "f64") is None


def test_width_predictor_chunks_respect_the_memory_budget():
    """bench.py's chunking for the batched tolerance mode: consecutive pairs,
    every pair once, at most `most` per chunk, and each chunk's output slots
    (from the library's plan, on the host) within the budget unless a single
    pair exceeds it on its own."""
    import torch
    import workloads as wk
    from paper_2410_04385_amd import api
    b = _bench()

    def cpu_tt(n, ranks):
        _, tot = api._offsets(n, ranks)
        return api.TT(torch.zeros(tot, dtype=torch.float64), n, ranks, 1)

    pairs = []
    for d, n, rx, ry in wk.batched_pair_shapes(7, 40):
        nn = [n] * d
        pairs.append((cpu_tt(nn, wk.feasible_ranks(nn, rx)), cpu_tt(nn, wk.feasible_ranks(nn, ry))))
    size = [8 * api.batched_adaptive_plan([p], 1e-6)["out_offset"][-1] for p in pairs]
    budget = 3 * max(size)
    chunks = b._rp_chunks(api, pairs, 1e-6, budget=budget, most=7)
    assert [k for ch in chunks for k in ch] == list(range(len(pairs)))
    assert all(1 <= len(ch) <= 7 for ch in chunks)
    assert all(sum(size[k] for k in ch) <= budget for ch in chunks)
    # a chunk closes only when the next pair would break a limit
    for ch, nxt in zip(chunks, chunks[1:]):
        assert len(ch) == 7 or sum(size[k] for k in ch) + size[nxt[0]] > budget
