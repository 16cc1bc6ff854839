"""A recompression step captured in a HIP graph (through torch's graph API
on the library's stream) replays to the same result as eager execution,
replay after replay, with eager work and synchronisations in between."""

import sys

import numpy as np
import pytest
import torch

import workloads as wk
import paper_2410_04385_amd as H

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    print("[gpu-case] graph capture of hatt_recompress, spectral d=8 batch 4", flush=True)
    pairs = [wk.spectral_pair(50 + b, d=8, n=16, rx=12, ry=10) for b in range(4)]
    x = H.TT.from_cores([p[0] for p in pairs])
    y = H.TT.from_cores([p[1] for p in pairs])
    p = H.plan(x, y, 24, max_rank=10, seed=3)
    out = H.TT.empty(x.n, p["ell"], 4)
    ranks = torch.empty((4, 9), dtype=torch.int64, device="cuda")
    ws = torch.empty(p["ws_bytes"], dtype=torch.uint8, device="cuda")

    def step():
        H.recompress(x, y, 24, max_rank=10, seed=3, workspace=ws, out=out, ranks=ranks)

    step()
    torch.cuda.synchronize()
    ref = out.data.clone()
    ref_r = ranks.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        out.data.fill_(0.0)
        ranks.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ranks, ref_r), rep
        assert torch.equal(out.data, ref), rep
        step()                      # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out.data, ref)


def test_uneven_batch_graph_replays_match_eager():
    print("[gpu-case] graph capture of hatt_recompress_batched, 12 uneven pairs on the library streams",
          flush=True)
    rng = np.random.default_rng(31)
    pairs = []
    for p in range(12):
        d = int(rng.integers(3, 9))
        n = int(rng.choice([4, 8, 16]))
        x, y = wk.spectral_pair(3100 + p, d=d, n=n, rx=int(rng.integers(3, 13)), ry=int(rng.integers(3, 13)))
        pairs.append((H.TT.from_cores([x]), H.TT.from_cores([y])))
    plan = H.batched_plan(pairs, 0, tol=1e-6, seed=41)
    ws = torch.empty(plan["ws_bytes"], dtype=torch.uint8, device="cuda")
    out = torch.zeros(plan["out_offset"][-1], dtype=torch.float64, device="cuda")
    ranks = torch.zeros(plan["rank_offset"][-1], dtype=torch.int64, device="cuda")

    def step():
        H.recompress_batched(pairs, 0, tol=1e-6, seed=41, workspace=ws, out=out, ranks=ranks)

    step()
    torch.cuda.synchronize()
    ref, ref_r = out.clone(), ranks.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(3):
        out.fill_(0.0)
        ranks.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ranks, ref_r), rep
        assert torch.equal(out, ref), rep
        step()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
