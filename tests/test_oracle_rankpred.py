"""Pins of the width predictor's oracle (oracle/rankpred.py): library
routines for the statistics, closed forms for spectral cores and for Adam,
central differences for the gradient, and properties of the widths."""

import math

import numpy as np
import pytest

import workloads as wk
from oracle import adapt, plan, rankpred as rp, tt


def _rng(s=0):
    return np.random.default_rng(s)


def test_quantiles_match_numpy_linear():
    g = _rng(1)
    for r in (1, 2, 3, 7, 8, 20, 48):
        v = g.standard_normal(r)
        ref = np.quantile(v, [j / 7 for j in range(8)])  # numpy's default: linear
        assert np.allclose(rp.quantiles8(v), ref, rtol=0, atol=1e-15)


def test_log_col_norms_match_numpy():
    core = _rng(2).standard_normal((5, 4, 7))
    ref = np.log(np.linalg.norm(core.reshape(20, 7), axis=0) ** 2)
    assert np.allclose(rp.log_col_norms(core), ref, rtol=1e-14, atol=0)
    z = np.zeros((2, 3, 2))
    assert rp.log_col_norms(z) == [math.log(1e-300)] * 2


def test_features_of_spectral_cores_closed_form():
    # V(core) = Q diag(2^(-j/2)), Q orthonormal: column norms^2 are 2^(-j)
    x, y = wk.spectral_pair(3, d=6, n=8, rx=5, ry=9)
    f = rp.features(x, y)
    assert f.shape == (5, 21)
    for k in range(1, 6):
        row = f[k - 1]
        rxk, ryk = tt.ranks(x)[k], tt.ranks(y)[k]
        assert row[0] == pytest.approx(math.log(rxk)) and row[1] == pytest.approx(math.log(ryk))
        assert row[2] == pytest.approx(math.log(8)) and row[3] == pytest.approx(k / 6)
        assert row[4] == pytest.approx(math.log(6))
        qx = np.quantile(-math.log(2) * np.arange(1, rxk + 1), [j / 7 for j in range(8)])
        qy = np.quantile(-math.log(2) * np.arange(1, ryk + 1), [j / 7 for j in range(8)])
        assert np.allclose(row[5:13], qx, atol=1e-12)
        assert np.allclose(row[13:21], qy, atol=1e-12)


def _net(seed=4, scale=0.5):
    g = _rng(seed)
    theta = g.standard_normal(rp.N_THETA) * scale
    stats = np.concatenate([g.standard_normal(21), 0.5 + g.random(21), g.standard_normal(2), 0.5 + g.random(2)])
    return theta, stats


def test_layout_sizes():
    assert rp.N_THETA == 19586 and rp.N_STATS == 46
    theta, _ = _net()
    assert np.array_equal(rp.pack(rp.unpack(theta)), theta)


def test_gradient_matches_central_differences():
    theta, stats = _net()
    g = _rng(5)
    feat = g.standard_normal((6, 21)) * 2
    lab = g.standard_normal((6, 2)) * 3
    L, grad = rp.loss_and_grad(theta, stats, feat, lab)
    # coordinates from every block, including the first and last of each
    offs, o = [], 0
    for _, shp in rp.SIZES:
        sz = int(np.prod(shp))
        offs += [o, o + sz - 1] + list(o + g.integers(0, sz, 3))
        o += sz
    h = 1e-6
    for i in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (rp.loss_and_grad(tp, stats, feat, lab)[0] - rp.loss_and_grad(tm, stats, feat, lab)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_loss_closed_form_with_silent_last_layer():
    theta, stats = _net()
    P = rp.unpack(theta)
    P["W3"][:] = 0.0
    P["b3"][:] = [0.25, -1.5]
    theta = rp.pack(P)
    feat = _rng(6).standard_normal((4, 21))
    pred = rp.predict(theta, stats, feat)
    my, sy = stats[42:44], stats[44:46]
    assert np.allclose(pred, np.array([0.25, -1.5]) * sy + my)
    lab = np.tile(my, (4, 1))  # standardised targets 0
    L, _ = rp.loss_and_grad(theta, stats, feat, lab)
    assert L == pytest.approx(0.5 * (0.25 ** 2 + 1.5 ** 2))


def test_adam_constant_gradient_steps_by_lr():
    # with a constant gradient the bias-corrected moments are g and g^2
    # exactly, so every step moves each coordinate by lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 6):
        th2, m, v = rp.adam(th, m, v, g, t, lr=0.01)
        assert np.allclose(th2 - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
        th = th2


def test_fit_stats_standardises():
    g = _rng(7)
    feat = g.standard_normal((50, 21)) * 3 + 2
    feat[:, 4] = 1.7  # constant column
    lab = g.standard_normal((50, 2)) + 5
    s = rp.fit_stats(feat, lab)
    z = (feat - s[:21]) / s[21:42]
    assert np.allclose(z.mean(0), 0, atol=1e-12)
    std = z.std(0)
    assert np.allclose(np.delete(std, 4), 1, atol=1e-12) and s[21 + 4] == 1.0 and np.all(np.abs(z[:, 4]) < 1e-14)


def test_training_reduces_loss():
    g = _rng(8)
    feat = g.standard_normal((256, 21))
    lab = np.stack([feat[:, 0] - 0.5 * feat[:, 3], np.tanh(feat[:, 1]) + feat[:, 2]], axis=1)
    stats = rp.fit_stats(feat, lab)
    theta = wk.mlp_init(9)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = rp.loss_and_grad(theta, stats, feat, lab)[0]
    for t in range(1, 201):
        idx = g.integers(0, 256, 64)
        _, gr = rp.loss_and_grad(theta, stats, feat[idx], lab[idx])
        theta, m, v = rp.adam(theta, m, v, gr, t, lr=3e-3)
    L1 = rp.loss_and_grad(theta, stats, feat, lab)[0]
    assert L1 < 0.1 * L0


def test_labels_and_widths():
    kept = [1, 12, 30, 30, 4, 1]
    cap = [1, 16, 64, 35, 4, 1]
    lab = rp.labels(kept, cap, p=8)
    assert np.allclose(np.exp(lab), [[12, 16], [30, 38], [30, 35], [4, 4]])
    n, rx, ry = [4, 4, 8, 8, 4], [1, 4, 8, 8, 2, 1], [1, 4, 8, 8, 2, 1]
    pred = np.log(np.array([[10.5, 17.2], [30.2, 37.1], [25.0, 20.0], [3.5, 40.0]]))
    ell, rho = rp.widths(pred, n, rx, ry, margin=0.0, p=8)
    req = [1, 19, 39, 33, 40, 1]  # ceil(max(e^b, e^a + 8))
    assert ell == plan.clamp_ell(n, rx, ry, req) and rho == [1, 11, 31, 25, 4, 1]
    ell2, _ = rp.widths(pred, n, rx, ry, margin=0.25, p=8)
    assert all(a >= b for a, b in zip(ell2, ell))
    big, _ = rp.widths(np.full((4, 2), 50.0), n, rx, ry, margin=0.0)
    assert big == plan.clamp_ell(n, rx, ry, [1 << 40] * 6)


def test_adaptive_started_at_accepted_widths_accepts_at_once():
    pairs = [wk.spectral_pair(11, d=5, n=4, rx=3, ry=4)]
    outs, ell, att, ok = adapt.hatt_adaptive(pairs, 1e-6, seed=2)
    assert ok and att >= 1
    outs2, ell2, att2, ok2 = adapt.hatt_adaptive(pairs, 1e-6, seed=2 + (att - 1), ell0=ell)
    assert ok2 and att2 == 1 and ell2 == ell
    assert tt.rel_err(outs2[0], outs[0]) < 1e-12
