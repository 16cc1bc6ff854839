"""The static-scratch entry point (hatt_recompress_noalloc) against the
workspace entry point (hatt_recompress) through the C ABI: two calls in a
row, the second on a smaller problem, each matching the workspace call to the
same bar as the parity tests (ranks exact, tensors within 1e-10)."""

import numpy as np
import pytest
import torch

import paper_2410_04385_amd as H
import workloads as wk
from oracle import tt

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _both(x, y, ell, **kw):
    p = H.plan(x, y, ell, **kw)
    assert p["ws_bytes"] <= 128 << 20
    a = H.recompress(x, y, ell, **kw)
    b = H.recompress_noalloc(x, y, ell, **kw)
    torch.cuda.synchronize()
    return a, b


def test_noalloc_matches_workspace_entry_point_twice():
    # first call: a batch of two spectral pairs, truncated by cap
    pairs = [wk.spectral_pair(700 + i, d=8, n=16, rx=12, ry=12) for i in range(2)]
    x = H.TT.from_cores([p[0] for p in pairs])
    y = H.TT.from_cores([p[1] for p in pairs])
    print("noalloc call 1: spectral d=8 n=16 r=12 ell=20 cap=10, batch 2", flush=True)
    a, b = _both(x, y, 20, max_rank=10, seed=5)
    for i in range(2):
        assert a.ranks[i].tolist() == b.ranks[i].tolist()
        assert tt.rel_err(b.train(i), a.train(i)) <= TOL
    # second call, smaller: the tiny pair at exact rank, no truncation
    yt, zt = wk.tiny_pair(3)
    print("noalloc call 2: tiny d=6 n=4 r=3 ell=9", flush=True)
    a2, b2 = _both(H.TT.from_cores(yt), H.TT.from_cores(zt), 9, seed=6)
    assert a2.ranks[0].tolist() == b2.ranks[0].tolist() == [1, 4, 9, 9, 9, 4, 1]
    assert tt.rel_err(b2.train(0), a2.train(0)) <= TOL
    full = tt.full(yt) * tt.full(zt)
    assert np.linalg.norm(tt.full(b2.train(0)) - full) <= 1e-12 * np.linalg.norm(full)
