"""Width predictor on the GPU against the FP64 oracle (oracle/rankpred.py):
core statistics, inference, the loss gradient, Adam, the standardisation,
and what the trained network gains over the adaptive method it starts."""

import math
import time

import numpy as np
import pytest
import torch

import workloads as wk
import paper_2410_04385_amd as H
from oracle import adapt, plan as oplan, rankpred as orp, tt

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _pairs_to_dev(pairs):
    return [(H.TT.from_cores([x]), H.TT.from_cores([y])) for x, y in pairs]


def _net(seed, scale=0.3):
    g = np.random.default_rng(seed)
    theta = g.standard_normal(orp.N_THETA) * scale
    stats = np.concatenate([g.standard_normal(21), 0.5 + g.random(21), g.standard_normal(2), 0.5 + g.random(2)])
    return theta, stats


def _f32(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")


def test_features_match_oracle():
    _say("rankpred features: uneven spectral/gaussian pairs, d up to 40, rank 300")
    g = np.random.default_rng(1)
    host = []
    for s in range(6):
        d = int(g.integers(2, 9))
        host.append(wk.spectral_pair(100 + s, d=d, n=int(g.choice([4, 8])), rx=int(g.integers(1, 9)),
                                     ry=int(g.integers(1, 9))))
    n = [2] * 40  # 39 bonds: two feature launches
    host.append((wk.gaussian_tt(g, n, wk.feasible_ranks(n, 5)), wk.gaussian_tt(g, n, wk.feasible_ranks(n, 3))))
    n = [300, 2, 300]  # bond rank 300: more columns than threads
    host.append((wk.gaussian_tt(g, n, [1, 300, 300, 1]), wk.gaussian_tt(g, n, [1, 7, 7, 1])))
    pairs = _pairs_to_dev(host)
    f = H.rankpred_features(pairs).cpu().numpy()
    ref = np.concatenate([orp.features(x, y) for x, y in host])
    assert f.shape == ref.shape == (H.rankpred_rows(pairs), 21)
    assert np.allclose(f, ref.astype(np.float32), rtol=2e-6, atol=2e-5)


def test_forward_matches_oracle():
    _say("rankpred forward: 1000 rows (ragged last block)")
    theta, stats = _net(2)
    feat = np.random.default_rng(3).standard_normal((1000, 21)) * 2
    pred = H.rankpred_forward(_f32(theta), _f32(stats), _f32(feat)).cpu().numpy()
    th32 = theta.astype(np.float32).astype(np.float64)
    st32 = stats.astype(np.float32).astype(np.float64)
    ref = orp.predict(th32, st32, feat.astype(np.float32).astype(np.float64))
    # FP32 network: inputs rounded identically, then ~130-term FP32 sums
    assert np.max(np.abs(pred - ref) / (1.0 + np.abs(ref))) < 2e-5


@pytest.mark.parametrize("batch", [1, 64, 150, 700])
def test_gradient_matches_oracle(batch):
    _say(f"rankpred gradient: batch {batch}")
    theta, stats = _net(4)
    g = np.random.default_rng(5)
    feat = g.standard_normal((400, 21)) * 2
    lab = g.standard_normal((400, 2)) * 3
    idx = g.integers(0, 400, batch).astype(np.int32)  # repeats allowed
    grad, loss = H.rankpred_grad(_f32(theta), _f32(stats), _f32(feat), _f32(lab),
                                 torch.tensor(idx, device="cuda"))
    f64 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    L, ref = orp.loss_and_grad(f64(theta), f64(stats), f64(feat)[idx], f64(lab)[idx])
    gg = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - L) <= 1e-5 * max(1.0, L)
    assert np.linalg.norm(gg - ref) <= 1e-5 * np.linalg.norm(ref)
    off = 0
    for name, shp in orp.SIZES:  # every block, not just the bulk
        sz = int(np.prod(shp))
        blk, rb = gg[off:off + sz], ref[off:off + sz]
        assert np.linalg.norm(blk - rb) <= 1e-4 * np.linalg.norm(rb) + 1e-7, name
        off += sz


def test_adam_step_matches_oracle():
    _say("rankpred Adam: three steps")
    theta, stats = _net(6)
    g = np.random.default_rng(7)
    feat = g.standard_normal((256, 21))
    lab = g.standard_normal((256, 2))
    th = _f32(theta)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    mh, vh, thh = np.zeros(orp.N_THETA), np.zeros(orp.N_THETA), th.cpu().numpy().astype(np.float64)
    F, Lb = _f32(feat), _f32(lab)
    for step in range(1, 4):
        idx = torch.tensor(g.integers(0, 256, 96).astype(np.int32), device="cuda")
        grad, _ = H.rankpred_grad(th, _f32(stats), F, Lb, idx)  # the gradient the step uses
        H.rankpred_train_step(th, m, v, step, _f32(stats), F, Lb, idx, lr=1e-2)
        thh, mh, vh = orp.adam(thh, mh, vh, grad.cpu().numpy().astype(np.float64), step, lr=1e-2)
        got = th.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - thh)) <= 1e-2 * 1e-4 + 1e-6 * np.max(np.abs(thh)), step
        thh = got  # keep the two sides on the same iterate


def test_fit_stats_match_oracle():
    _say("rankpred stats: 3000 rows, one constant column")
    g = np.random.default_rng(8)
    feat = (g.standard_normal((3000, 21)) * 3 + 1).astype(np.float32)
    feat[:, 4] = 2.5
    lab = (g.standard_normal((3000, 2)) + 4).astype(np.float32)
    s = H.rankpred_fit_stats(_f32(feat), _f32(lab)).cpu().numpy()
    ref = orp.fit_stats(feat.astype(np.float64), lab.astype(np.float64))
    assert np.allclose(s, ref, rtol=1e-6, atol=1e-6) and s[21 + 4] == 1.0


# ---------------------------------------------------------------------------
# What the network gains: small uneven pairs with the 2^(-j/2) spectrum at
# tol 1e-6, trained on the adaptive method's accepted kept ranks.

TOL = 1e-6


def _small_pairs(seed, count):
    g = np.random.default_rng(seed)
    out = []
    for p in range(count):
        d = int(g.integers(4, 7))
        n = int(g.choice([4, 8]))
        out.append(wk.spectral_pair(seed * 1000 + p, d=d, n=n, rx=int(g.integers(6, 17)), ry=int(g.integers(6, 17))))
    return out


def _adaptive(pair, seed, ell_init=None):
    X, Y = pair
    t0 = time.perf_counter()
    res, ell, att = H.recompress_adaptive(X, Y, TOL, seed=seed, ell_init=ell_init)
    torch.cuda.synchronize()
    return res, ell, att, time.perf_counter() - t0


def test_trained_predictor_saves_attempts():
    _say("rankpred gain: 40 training pairs, 12 fresh pairs, tol 1e-6")
    train_host = _small_pairs(21, 40)
    train = _pairs_to_dev(train_host)
    labels = []
    for i, pr in enumerate(train):
        res, ell, att, _ = _adaptive(pr, 500 + i)
        kept = res.ranks[0].cpu().tolist()
        x, y = pr
        cap = oplan.clamp_ell(x.n, x.ranks, y.ranks, [1 << 40] * (x.d + 1))
        labels.append(orp.labels(kept, cap, p=8))
    feat = H.rankpred_features(train)
    lab = _f32(np.concatenate(labels))
    stats = H.rankpred_fit_stats(feat, lab)
    theta = _f32(wk.mlp_init(3))
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    rows = feat.shape[0]
    g = np.random.default_rng(9)
    losses = []
    for step in range(1, 601):
        idx = torch.tensor(g.integers(0, rows, 64).astype(np.int32), device="cuda")
        losses.append(H.rankpred_train_step(theta, m, v, step, stats, feat, lab, idx, lr=3e-3))
    first, last = float(losses[0].item()), float(torch.stack(losses[-20:]).mean().item())
    assert last < 0.2 * first, (first, last)

    fresh_host = _small_pairs(77, 12)
    fresh = _pairs_to_dev(fresh_host)
    pred = H.rankpred_forward(theta, stats, H.rankpred_features(fresh))
    widths = H.rankpred_widths(fresh, pred, margin=0.1)
    att_plain, att_pred = [], []
    for i, (pr, hp) in enumerate(zip(fresh, fresh_host)):
        r0, ell0, a0, _ = _adaptive(pr, 900 + i)
        r1, ell1, a1, _ = _adaptive(pr, 900 + i, ell_init=widths[i][0])
        att_plain.append(a0)
        att_pred.append(a1)
        z = tt.full(hp[0]) * tt.full(hp[1])
        nz = np.linalg.norm(z)
        for res in (r0, r1):  # both results meet the tolerance against the exact product
            assert np.linalg.norm(tt.full(res.train(0)) - z) <= 3 * TOL * nz
    _say(f"attempts plain {att_plain} predicted {att_pred}")
    assert np.mean(att_pred) < np.mean(att_plain)
    assert sum(a == 1 for a in att_pred) >= 9


def test_rel_err_and_labels_match_oracle():
    _say("rel_err through the difference TT; labels")
    g = np.random.default_rng(12)
    for d in (1, 2, 5):
        n = [3] * d
        a = wk.gaussian_tt(g, n, wk.feasible_ranks(n, 4))
        b = [c + 1e-3 * g.standard_normal(c.shape) for c in a]
        da = [torch.tensor(c, device="cuda") for c in a]
        db = [torch.tensor(c, device="cuda") for c in b]
        assert H.rel_err(da, db) == pytest.approx(tt.rel_err(a, b), rel=1e-8)
    kept, cap = [1, 5, 20, 7, 1], [1, 8, 24, 7, 1]
    assert np.allclose(H.rankpred_labels(kept, cap), orp.labels(kept, cap).astype(np.float32))
