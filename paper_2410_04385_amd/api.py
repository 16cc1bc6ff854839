"""Python binding of libhatt: device memory and streams come from PyTorch;
every arithmetic step runs in the HIP library behind the C ABI."""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import HattAdamOpts, HattAdaptOpts, HattOpts, HattTT, check, i64_array, lib


def _offsets(n: Sequence[int], r: Sequence[int]):
    off, acc = [], 0
    for k in range(len(n)):
        off.append(acc)
        acc += int(r[k]) * int(n[k]) * int(r[k + 1])
    return off, acc


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class TT:
    """``batch`` tensor trains of identical shape in one flat float64 device
    tensor; core k of train b is the row-major block
    data[b*stride + off[k] : ...] of shape (rank[k], n[k], rank[k+1])."""

    def __init__(self, data: torch.Tensor, n: Sequence[int], ranks: Sequence[int], batch: int = 1,
                 stride: Optional[int] = None):
        self.n = [int(v) for v in n]
        self.ranks = [int(v) for v in ranks]
        self.d = len(self.n)
        self.batch = int(batch)
        self.off, self.total = _offsets(self.n, self.ranks)
        self.stride = int(stride) if stride else self.total
        if data.dtype != torch.float64 or data.dim() != 1:
            raise ValueError("TT data must be a flat float64 tensor")
        if data.numel() < (self.batch - 1) * self.stride + self.total:
            raise ValueError("TT data too small for its shape")
        self.data = data

    @staticmethod
    def empty(n, ranks, batch=1, device="cuda") -> "TT":
        _, tot = _offsets(n, ranks)
        return TT(torch.zeros(batch * tot, dtype=torch.float64, device=device), n, ranks, batch)

    @staticmethod
    def from_cores(trains, device="cuda") -> "TT":
        """``trains``: one TT (list of arrays) or a list of TTs of one shape."""
        if isinstance(trains[0], np.ndarray) or torch.is_tensor(trains[0]):
            trains = [trains]
        n = [int(c.shape[1]) for c in trains[0]]
        ranks = [int(trains[0][0].shape[0])] + [int(c.shape[2]) for c in trains[0]]
        flat = []
        for t in trains:
            if [int(c.shape[1]) for c in t] != n:
                raise ValueError("trains differ in shape")
            for c in t:
                flat.append(np.ascontiguousarray(np.asarray(c, dtype=np.float64)).ravel())
        host = torch.from_numpy(np.concatenate(flat))
        return TT(host.to(device), n, ranks, len(trains))

    @staticmethod
    def from_device_cores(cores: Sequence[torch.Tensor]) -> "TT":
        """One train from device cores (r_k, n_k, r_{k+1}), packed into a flat
        buffer (a device copy)."""
        n = [int(c.shape[1]) for c in cores]
        ranks = [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]
        data = torch.cat([c.reshape(-1) for c in cores]).to(torch.float64).contiguous()
        return TT(data, n, ranks, 1)

    def view(self):
        n_arr, r_arr = i64_array(self.n), i64_array(self.ranks)
        v = HattTT(self.d, self.batch, n_arr, r_arr, ctypes.c_void_p(self.data.data_ptr()), self.stride)
        return v, (n_arr, r_arr)

    def core(self, k: int, b: int = 0) -> torch.Tensor:
        s = b * self.stride + self.off[k]
        e = s + self.ranks[k] * self.n[k] * self.ranks[k + 1]
        return self.data[s:e].view(self.ranks[k], self.n[k], self.ranks[k + 1])

    def to_numpy(self, b: int = 0, kept: Optional[Sequence[int]] = None) -> List[np.ndarray]:
        out = []
        for k in range(self.d):
            c = self.core(k, b).detach().cpu().numpy()
            if kept is not None:
                c = c[: int(kept[k]), :, : int(kept[k + 1])]
            out.append(np.array(c))
        return out


@dataclass
class Result:
    out: TT                  # capacity-shape cores
    ranks: torch.Tensor      # device int64 [batch, d+1]

    def train(self, b: int = 0) -> List[np.ndarray]:
        kept = self.ranks[b].cpu().tolist()
        return self.out.to_numpy(b, kept)


_PRECISION = {"f64": 0, "f32": 1, "bf16": 2}


def _opts(ell, max_rank, tol, seed, variant, ep, d, precision="f64"):
    ell_arr = None
    if not np.isscalar(ell):
        if len(ell) != d + 1:
            raise ValueError("per-bond ell needs d+1 entries")
        ell_arr = i64_array(ell)
        ell_u = 0
    else:
        ell_u = int(ell)
    if precision not in _PRECISION:
        raise ValueError(f"precision must be one of {sorted(_PRECISION)}")
    mr_arr = None
    if np.isscalar(max_rank):
        mr_u = int(max_rank)
    else:
        # per-bond caps: entry k caps bond k (<= 0: no cap there)
        if len(max_rank) != d + 1:
            raise ValueError("per-bond max_rank needs d+1 entries")
        mr_arr = i64_array(max_rank)
        mr_u = 0
    o = HattOpts(int(variant), float(ep), ell_u, ell_arr, mr_u, float(tol), int(seed) & 0xFFFFFFFFFFFFFFFF,
                 _PRECISION[precision], mr_arr)
    return o, (ell_arr, mr_arr)


def plan(x: TT, y: TT, ell, max_rank: int = 0, tol: float = 0.0, seed: int = 0, variant: int = 1,
         ep: float = 0.0, precision: str = "f64"):
    xv, kx = x.view()
    yv, ky = y.view()
    o, ka = _opts(ell, max_rank, tol, seed, variant, ep, x.d, precision)
    ell_out = (ctypes.c_int64 * (x.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("hatt_plan", lib().hatt_plan(ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(o), ell_out,
                                       ctypes.byref(ws), ctypes.byref(oe)))
    return {"ell": list(ell_out), "ws_bytes": int(ws.value), "out_elems": int(oe.value)}


def recompress(x: TT, y: TT, ell, *, max_rank: int = 0, tol: float = 0.0, seed: int = 0,
               sketch: Optional[TT] = None, variant: int = 1, ep: float = 0.0, precision: str = "f64",
               workspace: Optional[torch.Tensor] = None, out: Optional[TT] = None,
               ranks: Optional[torch.Tensor] = None, stream=None) -> Result:
    """HaTT (Alg. 4) of x (.) y for every train of the batch, optionally
    truncated by TT-Rounding to ``max_rank`` / ``tol``.  precision "f32" /
    "bf16": range finding on the FP32 / BF16 matrix cores, projection and
    truncation in FP64."""
    p = plan(x, y, ell, max_rank, tol, seed, variant, ep, precision)
    dev = x.data.device
    if out is None:
        out = TT.empty(x.n, p["ell"], x.batch, device=dev)
    if ranks is None:
        ranks = torch.empty((x.batch, x.d + 1), dtype=torch.int64, device=dev)
    if workspace is None or workspace.numel() < p["ws_bytes"]:
        workspace = torch.empty(max(p["ws_bytes"], 1), dtype=torch.uint8, device=dev)
    xv, kx = x.view()
    yv, ky = y.view()
    o, ka = _opts(ell, max_rank, tol, seed, variant, ep, x.d, precision)
    sk_ptr = None
    keep = None
    if sketch is not None:
        sv, keep = sketch.view()
        sk_ptr = ctypes.byref(sv)
    st = lib().hatt_recompress(ctypes.byref(xv), ctypes.byref(yv), sk_ptr, ctypes.byref(o),
                               ctypes.c_void_p(out.data.data_ptr()), out.stride,
                               ctypes.c_void_p(ranks.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                               workspace.numel(), _stream_ptr(stream))
    check("hatt_recompress", st)
    return Result(out, ranks)


def recompress_noalloc(x: TT, y: TT, ell, *, max_rank: int = 0, tol: float = 0.0, seed: int = 0,
                       sketch: Optional[TT] = None, variant: int = 1, ep: float = 0.0, precision: str = "f64",
                       out: Optional[TT] = None, ranks: Optional[torch.Tensor] = None, stream=None) -> Result:
    """recompress() on the library's static scratch array (no workspace):
    for problems whose workspace fits in 128 MiB."""
    p = plan(x, y, ell, max_rank, tol, seed, variant, ep, precision)
    dev = x.data.device
    if out is None:
        out = TT.empty(x.n, p["ell"], x.batch, device=dev)
    if ranks is None:
        ranks = torch.empty((x.batch, x.d + 1), dtype=torch.int64, device=dev)
    xv, kx = x.view()
    yv, ky = y.view()
    o, ka = _opts(ell, max_rank, tol, seed, variant, ep, x.d, precision)
    sk_ptr = None
    keep = None
    if sketch is not None:
        sv, keep = sketch.view()
        sk_ptr = ctypes.byref(sv)
    st = lib().hatt_recompress_noalloc(ctypes.byref(xv), ctypes.byref(yv), sk_ptr, ctypes.byref(o),
                                       ctypes.c_void_p(out.data.data_ptr()), out.stride,
                                       ctypes.c_void_p(ranks.data_ptr()), _stream_ptr(stream))
    check("hatt_recompress_noalloc", st)
    return Result(out, ranks)


def batched_plan(pairs, ell: int = 0, *, max_rank: int = 0, tol: float = 0.0, seed: int = 0, variant: int = 1,
                 ep: float = 0.0, precision: str = "f64"):
    """Plan of recompress_batched: per-pair output and rank offsets, widths,
    workspace bytes."""
    npairs = len(pairs)
    views = [(x.view(), y.view()) for x, y in pairs]
    xs = (HattTT * npairs)(*[v[0][0] for v in views])
    ys = (HattTT * npairs)(*[v[1][0] for v in views])
    o, _ = _opts(int(ell), max_rank, tol, seed, variant, ep, 0, precision)
    oo = (ctypes.c_int64 * (npairs + 1))()
    ro = (ctypes.c_int64 * (npairs + 1))()
    ne = sum(x.d + 1 for x, _ in pairs)
    eo = (ctypes.c_int64 * ne)()
    ws = ctypes.c_size_t(0)
    check("hatt_batched_plan", lib().hatt_batched_plan(npairs, xs, ys, ctypes.byref(o), oo, ro, eo,
                                                       ctypes.byref(ws)))
    ells, e = [], 0
    for x, _ in pairs:
        ells.append(list(eo[e:e + x.d + 1]))
        e += x.d + 1
    return {"out_offset": list(oo), "rank_offset": list(ro), "ell": ells, "ws_bytes": int(ws.value),
            "_keep": (views, xs, ys)}


def recompress_batched(pairs, ell: int = 0, *, max_rank: int = 0, tol: float = 0.0, seed: int = 0,
                       variant: int = 1, ep: float = 0.0, precision: str = "f64",
                       workspace: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                       ranks: Optional[torch.Tensor] = None, stream=None) -> List[Result]:
    """Uneven batch: ``pairs`` is a list of (x, y) TT pairs of any shapes;
    pair p uses the sketch keyed by seed + p; ell <= 0 asks for
    l_k = max(r_k, s_k) + 8.  ``out`` / ``ranks`` (flat float64 / int64
    device tensors of at least out_offset[-1] / rank_offset[-1] elements of
    batched_plan) may be passed in, e.g. for graph capture.  ``precision``
    "f32" / "bf16": every pair's HPCRL on the FP32 / BF16 matrix cores, the
    sweep and truncation in FP64.  Returns one Result per pair (views into one
    output buffer)."""
    p = batched_plan(pairs, ell, max_rank=max_rank, tol=tol, seed=seed, variant=variant, ep=ep,
                     precision=precision)
    views, xs, ys = p["_keep"]
    dev = pairs[0][0].data.device
    if out is None:
        out = torch.zeros(max(p["out_offset"][-1], 1), dtype=torch.float64, device=dev)
    elif out.dtype != torch.float64 or out.numel() < p["out_offset"][-1]:
        raise ValueError("out must be float64 with out_offset[-1] elements")
    if ranks is None:
        ranks = torch.empty(max(p["rank_offset"][-1], 1), dtype=torch.int64, device=dev)
    elif ranks.dtype != torch.int64 or ranks.numel() < p["rank_offset"][-1]:
        raise ValueError("ranks must be int64 with rank_offset[-1] elements")
    if workspace is None or workspace.numel() < p["ws_bytes"]:
        workspace = torch.empty(max(p["ws_bytes"], 1), dtype=torch.uint8, device=dev)
    o, _ = _opts(int(ell), max_rank, tol, seed, variant, ep, 0, precision)
    check("hatt_recompress_batched", lib().hatt_recompress_batched(
        len(pairs), xs, ys, ctypes.byref(o), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ranks.data_ptr()),
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr(stream)))
    res = []
    for k, (x, _) in enumerate(pairs):
        a, b = p["out_offset"][k], p["out_offset"][k + 1]
        tt = TT(out[a:b], x.n, p["ell"][k], x.batch)
        ra, rb = p["rank_offset"][k], p["rank_offset"][k + 1]
        res.append(Result(tt, ranks[ra:rb].view(x.batch, x.d + 1)))
    return res


def recompress_adaptive(x: TT, y: TT, tol: float, *, seed: int = 0, oversample: int = 8,
                        max_attempts: int = 8, variant: int = 1, ep: float = 0.0,
                        ell_init: Optional[Sequence[int]] = None, precision: str = "f64",
                        workspace: Optional[torch.Tensor] = None, stream=None):
    """Tolerance-driven HaTT: grows the sketch widths until the truncation
    at ``tol`` leaves slack on every bond, starting from ``ell_init`` (d+1
    widths, e.g. predicted ones) or from max(r_k, s_k) + oversample.
    ``precision`` "f32" / "bf16": HPCRL sketches on the FP32 / BF16 matrix
    cores.
    Returns (Result, widths used, attempts)."""
    xv, kx = x.view()
    yv, ky = y.view()
    init = None
    if ell_init is not None:
        if len(ell_init) != x.d + 1:
            raise ValueError("ell_init needs d+1 entries")
        init = i64_array(ell_init)
    if precision not in _PRECISION:
        raise ValueError(f"unknown precision {precision!r}")
    o = HattAdaptOpts(float(tol), int(seed) & 0xFFFFFFFFFFFFFFFF, int(oversample), int(max_attempts),
                      int(variant), float(ep), init, _PRECISION[precision])
    cap = (ctypes.c_int64 * (x.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("hatt_adaptive_plan", lib().hatt_adaptive_plan(ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(o),
                                                         cap, ctypes.byref(ws), ctypes.byref(oe)))
    dev = x.data.device
    slot = int(oe.value)
    data = torch.zeros(x.batch * slot, dtype=torch.float64, device=dev)
    ranks = torch.empty((x.batch, x.d + 1), dtype=torch.int64, device=dev)
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)
    ell = (ctypes.c_int64 * (x.d + 1))()
    att = ctypes.c_int32(0)
    check("hatt_recompress_adaptive", lib().hatt_recompress_adaptive(
        ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(o), ctypes.c_void_p(data.data_ptr()), slot,
        ctypes.c_void_p(ranks.data_ptr()), ell, ctypes.byref(att), ctypes.c_void_p(workspace.data_ptr()),
        workspace.numel(), _stream_ptr(stream)))
    out = TT(data, x.n, list(ell), x.batch, stride=slot)
    return Result(out, ranks), list(ell), int(att.value)


def _batched_adapt_opts(pairs, tol, seed, oversample, max_attempts, variant, ep, ell_init, precision):
    init = None
    if ell_init is not None:
        if len(ell_init) != len(pairs) or any(len(e) != x.d + 1 for e, (x, _) in zip(ell_init, pairs)):
            raise ValueError("ell_init needs d_p+1 widths for every pair")
        init = i64_array([v for e in ell_init for v in e])
    if precision not in _PRECISION:
        raise ValueError(f"unknown precision {precision!r}")
    o = HattAdaptOpts(float(tol), int(seed) & 0xFFFFFFFFFFFFFFFF, int(oversample), int(max_attempts),
                      int(variant), float(ep), init, _PRECISION[precision])
    return o, init


def batched_adaptive_plan(pairs, tol: float, *, seed: int = 0, oversample: int = 8, max_attempts: int = 8,
                          variant: int = 1, ep: float = 0.0, ell_init=None, precision: str = "f64"):
    """Plan of recompress_batched_adaptive: per-pair output and rank offsets,
    the widths each pair may grow to, and the smallest / full-concurrency
    workspace sizes."""
    npairs = len(pairs)
    views = [(x.view(), y.view()) for x, y in pairs]
    xs = (HattTT * npairs)(*[v[0][0] for v in views])
    ys = (HattTT * npairs)(*[v[1][0] for v in views])
    o, init = _batched_adapt_opts(pairs, tol, seed, oversample, max_attempts, variant, ep, ell_init, precision)
    oo = (ctypes.c_int64 * (npairs + 1))()
    ro = (ctypes.c_int64 * (npairs + 1))()
    co = (ctypes.c_int64 * sum(x.d + 1 for x, _ in pairs))()
    wmin, wfull = ctypes.c_size_t(0), ctypes.c_size_t(0)
    check("hatt_batched_adaptive_plan", lib().hatt_batched_adaptive_plan(
        npairs, xs, ys, ctypes.byref(o), oo, ro, co, ctypes.byref(wmin), ctypes.byref(wfull)))
    caps, e = [], 0
    for x, _ in pairs:
        caps.append(list(co[e:e + x.d + 1]))
        e += x.d + 1
    return {"out_offset": list(oo), "rank_offset": list(ro), "cap": caps, "ws_min": int(wmin.value),
            "ws_full": int(wfull.value), "_keep": (views, xs, ys, o, init)}


def recompress_batched_adaptive(pairs, tol: float, *, seed: int = 0, oversample: int = 8, max_attempts: int = 8,
                                variant: int = 1, ep: float = 0.0, ell_init=None, precision: str = "f64",
                                max_workspace: int = 64 << 30, workspace: Optional[torch.Tensor] = None,
                                stream=None):
    """Tolerance mode over an uneven batch: pair p follows recompress_adaptive
    with seed + p and its own widths; every attempt round runs the pairs not
    yet accepted side by side and synchronises once.  The workspace (given,
    or allocated at the full-concurrency size capped by ``max_workspace`` but
    never below the minimum) decides how many pairs run side by side.
    Returns (one Result per pair, widths per pair, attempts per pair)."""
    p = batched_adaptive_plan(pairs, tol, seed=seed, oversample=oversample, max_attempts=max_attempts,
                              variant=variant, ep=ep, ell_init=ell_init, precision=precision)
    views, xs, ys, o, _ = p["_keep"]
    dev = pairs[0][0].data.device
    out = torch.zeros(max(p["out_offset"][-1], 1), dtype=torch.float64, device=dev)
    ranks = torch.empty(max(p["rank_offset"][-1], 1), dtype=torch.int64, device=dev)
    if workspace is None:
        workspace = torch.empty(max(p["ws_min"], min(p["ws_full"], int(max_workspace))), dtype=torch.uint8,
                                device=dev)
    npairs = len(pairs)
    ell = (ctypes.c_int64 * sum(x.d + 1 for x, _ in pairs))()
    att = (ctypes.c_int32 * npairs)()
    check("hatt_recompress_batched_adaptive", lib().hatt_recompress_batched_adaptive(
        npairs, xs, ys, ctypes.byref(o), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ranks.data_ptr()), ell,
        att, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr(stream)))
    res, ells, e = [], [], 0
    for k, (x, _) in enumerate(pairs):
        a, b = p["out_offset"][k], p["out_offset"][k + 1]
        ells.append(list(ell[e:e + x.d + 1]))
        e += x.d + 1
        tt = TT(out[a:b], x.n, ells[-1], x.batch, stride=(b - a) // x.batch)
        ra, rb = p["rank_offset"][k], p["rank_offset"][k + 1]
        res.append(Result(tt, ranks[ra:rb].view(x.batch, x.d + 1)))
    return res, ells, list(att)


def plan3(x: TT, y: TT, w: TT, ell, max_rank: int = 0, tol: float = 0.0, seed: int = 0):
    """Widths, workspace and output size of recompress3."""
    xv, kx = x.view()
    yv, ky = y.view()
    wv, kw = w.view()
    o, ka = _opts(ell, max_rank, tol, seed, 1, 0.0, x.d)
    ell_out = (ctypes.c_int64 * (x.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("hatt_plan3", lib().hatt_plan3(ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(wv), ctypes.byref(o),
                                         ell_out, ctypes.byref(ws), ctypes.byref(oe)))
    return {"ell": list(ell_out), "ws_bytes": int(ws.value), "out_elems": int(oe.value)}


def recompress3(x: TT, y: TT, w: TT, ell, *, max_rank: int = 0, tol: float = 0.0, seed: int = 0,
                sketch: Optional[TT] = None, workspace: Optional[torch.Tensor] = None, stream=None) -> Result:
    """HaTT of the three-factor product x (.) y (.) w in one pass (three-mode
    products in place of the three-way PKP cores), optionally truncated to
    ``max_rank`` / ``tol``; one triple (batch 1), FP64, HaTT-1."""
    p = plan3(x, y, w, ell, max_rank, tol, seed)
    dev = x.data.device
    out = TT.empty(x.n, p["ell"], 1, device=dev)
    ranks = torch.empty((1, x.d + 1), dtype=torch.int64, device=dev)
    if workspace is None or workspace.numel() < p["ws_bytes"]:
        workspace = torch.empty(max(p["ws_bytes"], 1), dtype=torch.uint8, device=dev)
    xv, kx = x.view()
    yv, ky = y.view()
    wv, kw = w.view()
    o, ka = _opts(ell, max_rank, tol, seed, 1, 0.0, x.d)
    sk_ptr = None
    keep = None
    if sketch is not None:
        sv, keep = sketch.view()
        sk_ptr = ctypes.byref(sv)
    check("hatt_recompress3", lib().hatt_recompress3(
        ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(wv), sk_ptr, ctypes.byref(o),
        ctypes.c_void_p(out.data.data_ptr()), out.stride, ctypes.c_void_p(ranks.data_ptr()),
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr(stream)))
    return Result(out, ranks)


def recompress3_adaptive(x: TT, y: TT, w: TT, tol: float, *, seed: int = 0, oversample: int = 8,
                         max_attempts: int = 8, ell_init: Optional[Sequence[int]] = None,
                         workspace: Optional[torch.Tensor] = None, stream=None):
    """Tolerance-driven three-factor HaTT (the rule of recompress_adaptive,
    starting from max(r_k, s_k, t_k) + oversample).  Returns (Result, widths
    used, attempts)."""
    xv, kx = x.view()
    yv, ky = y.view()
    wv, kw = w.view()
    init = None
    if ell_init is not None:
        if len(ell_init) != x.d + 1:
            raise ValueError("ell_init needs d+1 entries")
        init = i64_array(ell_init)
    o = HattAdaptOpts(float(tol), int(seed) & 0xFFFFFFFFFFFFFFFF, int(oversample), int(max_attempts), 1, 0.0,
                      init, 0)
    cap = (ctypes.c_int64 * (x.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("hatt_adaptive_plan3", lib().hatt_adaptive_plan3(ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(wv),
                                                           ctypes.byref(o), cap, ctypes.byref(ws),
                                                           ctypes.byref(oe)))
    dev = x.data.device
    slot = int(oe.value)
    data = torch.zeros(slot, dtype=torch.float64, device=dev)
    ranks = torch.empty((1, x.d + 1), dtype=torch.int64, device=dev)
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)
    ell = (ctypes.c_int64 * (x.d + 1))()
    att = ctypes.c_int32(0)
    check("hatt_recompress3_adaptive", lib().hatt_recompress3_adaptive(
        ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(wv), ctypes.byref(o), ctypes.c_void_p(data.data_ptr()),
        slot, ctypes.c_void_p(ranks.data_ptr()), ell, ctypes.byref(att), ctypes.c_void_p(workspace.data_ptr()),
        workspace.numel(), _stream_ptr(stream)))
    out = TT(data, x.n, list(ell), 1, stride=slot)
    return Result(out, ranks), list(ell), int(att.value)


def hadamard_norm2(x: TT, y: TT, workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """||x (.) y||_F^2 per train (device float64 [batch]) by the PKP-free Gram
    recursion."""
    xv, kx = x.view()
    yv, ky = y.view()
    ws = ctypes.c_size_t(0)
    check("hatt_hadamard_norm2_plan", lib().hatt_hadamard_norm2_plan(ctypes.byref(xv), ctypes.byref(yv),
                                                                     ctypes.byref(ws)))
    dev = x.data.device
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)
    out = torch.empty(x.batch, dtype=torch.float64, device=dev)
    check("hatt_hadamard_norm2", lib().hatt_hadamard_norm2(
        ctypes.byref(xv), ctypes.byref(yv), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
        workspace.numel(), _stream_ptr(stream)))
    return out


def hadamard_explicit(x: TT, y: TT, out: Optional[TT] = None, stream=None) -> TT:
    """Explicit PKP cores of x (.) y (ranks r_k s_k)."""
    rr = [a * b for a, b in zip(x.ranks, y.ranks)]
    if out is None:
        out = TT.empty(x.n, rr, x.batch, device=x.data.device)
    xv, kx = x.view()
    yv, ky = y.view()
    check("tt_hadamard_explicit", lib().tt_hadamard_explicit(
        ctypes.byref(xv), ctypes.byref(yv), ctypes.c_void_p(out.data.data_ptr()), out.stride,
        _stream_ptr(stream)))
    return out


def randorth(a: TT, ell, *, max_rank: int = 0, tol: float = 0.0, seed: int = 0, sketch: Optional[TT] = None,
             workspace: Optional[torch.Tensor] = None, stream=None) -> Result:
    """RandOrth (Alg. 2) of an explicit TT, e.g. the PKP cores of
    hadamard_explicit(x, y), optionally truncated by TT-Rounding."""
    ell_arr = None if np.isscalar(ell) else i64_array(ell)
    ell_u = int(ell) if np.isscalar(ell) else 0
    av, ka = a.view()
    eo = (ctypes.c_int64 * (a.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("tt_randorth_plan", lib().tt_randorth_plan(ctypes.byref(av), ell_u, ell_arr, eo, ctypes.byref(ws),
                                                     ctypes.byref(oe)))
    dev = a.data.device
    out = TT.empty(a.n, list(eo), a.batch, device=dev)
    ranks = torch.empty((a.batch, a.d + 1), dtype=torch.int64, device=dev)
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)
    sk_ptr = None
    keep = None
    if sketch is not None:
        sv, keep = sketch.view()
        sk_ptr = ctypes.byref(sv)
    check("tt_randorth", lib().tt_randorth(ctypes.byref(av), sk_ptr, ell_u, ell_arr, int(seed) & 0xFFFFFFFFFFFFFFFF,
                                           int(max_rank), float(tol), ctypes.c_void_p(out.data.data_ptr()), out.stride,
                                           ctypes.c_void_p(ranks.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                           workspace.numel(), _stream_ptr(stream)))
    return Result(out, ranks)


def check_finite(a: TT, stream=None) -> torch.Tensor:
    """Device int32 [batch]: 1 where every entry of the train is finite."""
    flag = torch.empty(a.batch, dtype=torch.int32, device=a.data.device)
    av, ka = a.view()
    check("tt_check_finite", lib().tt_check_finite(ctypes.byref(av), ctypes.c_void_p(flag.data_ptr()),
                                                   _stream_ptr(stream)))
    return flag


def scale(a: TT, alpha: torch.Tensor, invert: bool = False, stream=None) -> TT:
    """In place: train b of ``a`` times alpha[b] (divided by it with
    invert); alpha is a float64 device tensor of length batch."""
    if alpha.dtype != torch.float64 or alpha.numel() < a.batch:
        raise ValueError("alpha must be float64 with batch entries")
    av, ka = a.view()
    check("tt_scale", lib().tt_scale(ctypes.byref(av), ctypes.c_void_p(alpha.data_ptr()), int(bool(invert)),
                                     _stream_ptr(stream)))
    return a


def round_plan(a: TT):
    av, ka = a.view()
    cap = (ctypes.c_int64 * (a.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("tt_round_plan", lib().tt_round_plan(ctypes.byref(av), cap, ctypes.byref(ws), ctypes.byref(oe)))
    return {"cap": list(cap), "ws_bytes": int(ws.value), "out_elems": int(oe.value)}


def round(a: TT, max_rank: int = 0, tol: float = 0.0, *, workspace: Optional[torch.Tensor] = None,
          stream=None) -> Result:  # noqa: A001 - mirrors the C name tt_round
    """TT-Rounding (Alg. 1) of every train."""
    p = round_plan(a)
    dev = a.data.device
    out = TT.empty(a.n, p["cap"], a.batch, device=dev)
    ranks = torch.empty((a.batch, a.d + 1), dtype=torch.int64, device=dev)
    if workspace is None or workspace.numel() < p["ws_bytes"]:
        workspace = torch.empty(max(p["ws_bytes"], 1), dtype=torch.uint8, device=dev)
    av, ka = a.view()
    check("tt_round", lib().tt_round(ctypes.byref(av), int(max_rank), float(tol),
                                     ctypes.c_void_p(out.data.data_ptr()), out.stride,
                                     ctypes.c_void_p(ranks.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel(), _stream_ptr(stream)))
    return Result(out, ranks)


def norm(a: TT, *, workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Frobenius norms (device tensor of length batch)."""
    av, ka = a.view()
    ws = ctypes.c_size_t(0)
    check("tt_norm_plan", lib().tt_norm_plan(ctypes.byref(av), ctypes.byref(ws)))
    dev = a.data.device
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(max(ws.value, 1), dtype=torch.uint8, device=dev)
    out = torch.empty(a.batch, dtype=torch.float64, device=dev)
    check("tt_norm", lib().tt_norm(ctypes.byref(av), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   _stream_ptr(stream)))
    return out


def sketch_fill(seed: int, n: Sequence[int], ell: Sequence[int], device="cuda", stream=None) -> TT:
    """The seeded random Gaussian TT of Def. 2.1 (Philox4x32-10)."""
    t = TT.empty(n, ell, 1, device=device)
    check("hatt_sketch_fill", lib().hatt_sketch_fill(int(seed) & 0xFFFFFFFFFFFFFFFF, len(n), i64_array(n),
                                                     i64_array(ell), ctypes.c_void_p(t.data.data_ptr()),
                                                     _stream_ptr(stream)))
    return t


def profile_start() -> None:
    check("hatt_profile_start", lib().hatt_profile_start())


def profile_stop() -> dict:
    """Per kernel class: (milliseconds summed over launches, launcher calls)."""
    n = _lib.PROFILE_CLASSES
    ms = (ctypes.c_double * n)()
    calls = (ctypes.c_int64 * n)()
    check("hatt_profile_stop", lib().hatt_profile_stop(ms, calls))
    return {lib().hatt_profile_class_name(i).decode(): (float(ms[i]), int(calls[i])) for i in range(n)}


def profile_report() -> str:
    """Per-launch-site table of the last profile_stop()."""
    return lib().hatt_profile_report().decode()


def set_qr_method(method: str) -> None:
    """"cholqr2" (default: CholeskyQR2 with per-pair Householder fallback) or
    "householder" (TSQR everywhere).  Plan again afterwards."""
    codes = {"cholqr2": 0, "householder": 1}
    if method not in codes:
        raise ValueError(f"unknown QR method {method!r}")
    check("hatt_set_qr_method", lib().hatt_set_qr_method(codes[method]))


_TUNE = {"off": 0, "record": 1, "use": 2}


def tune(mode: str) -> None:
    """Autotuner mode: "off" (fixed rules), "record" (time the candidates of
    each new shape bucket on first use, keep the fastest) or "use" (recorded
    choices only)."""
    if mode not in _TUNE:
        raise ValueError(f"tune mode must be one of {sorted(_TUNE)}")
    check("hatt_tune_mode", lib().hatt_tune_mode(_TUNE[mode]))


def tune_clear() -> None:
    check("hatt_tune_clear", lib().hatt_tune_clear())


def tune_table() -> str:
    """The recorded choices, one shape bucket per line."""
    need = int(lib().hatt_tune_table(None, 0))
    buf = ctypes.create_string_buffer(need)
    lib().hatt_tune_table(buf, need)
    return buf.value.decode()


def version() -> str:
    return lib().hatt_version().decode()


# ---------------------------------------------------------------------------
# Learned start widths (hatt_rankpred_*): FP32 device tensors in and out.

def _f32(t: torch.Tensor, name: str, numel: Optional[int] = None) -> ctypes.c_void_p:
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs {numel} elements")
    return ctypes.c_void_p(t.data_ptr())


def _pair_views(pairs):
    views = [(x.view(), y.view()) for x, y in pairs]
    xs = (HattTT * len(pairs))(*[v[0][0] for v in views])
    ys = (HattTT * len(pairs))(*[v[1][0] for v in views])
    return views, xs, ys


def rankpred_rows(pairs) -> int:
    return sum(x.d - 1 for x, _ in pairs)


def rankpred_features(pairs, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """[rows, 21] statistics of every bond of every pair (train 0)."""
    rows = rankpred_rows(pairs)
    dev = pairs[0][0].data.device
    if out is None:
        out = torch.empty((max(rows, 1), _lib.RANKPRED_NIN), dtype=torch.float32, device=dev)
    keep, xs, ys = _pair_views(pairs)
    check("hatt_rankpred_features", lib().hatt_rankpred_features(
        len(pairs), xs, ys, _f32(out, "out", rows * _lib.RANKPRED_NIN), _stream_ptr(stream)))
    return out[:rows]


def rankpred_fit_stats(feat: torch.Tensor, label: torch.Tensor, stream=None) -> torch.Tensor:
    stats = torch.empty(_lib.RANKPRED_NSTATS, dtype=torch.float32, device=feat.device)
    rows = feat.shape[0]
    check("hatt_rankpred_fit_stats", lib().hatt_rankpred_fit_stats(
        _f32(feat, "feat", rows * 21), _f32(label, "label", rows * 2), rows, _f32(stats, "stats"),
        _stream_ptr(stream)))
    return stats


def rankpred_forward(theta: torch.Tensor, stats: torch.Tensor, feat: torch.Tensor, stream=None) -> torch.Tensor:
    rows = feat.shape[0]
    pred = torch.empty((max(rows, 1), 2), dtype=torch.float32, device=feat.device)
    check("hatt_rankpred_forward", lib().hatt_rankpred_forward(
        _f32(theta, "theta", _lib.RANKPRED_NTHETA), _f32(stats, "stats", _lib.RANKPRED_NSTATS),
        _f32(feat, "feat", rows * 21), rows, _f32(pred, "pred"), _stream_ptr(stream)))
    return pred[:rows]


def _idx(idx: torch.Tensor) -> ctypes.c_void_p:
    if idx.dtype != torch.int32 or not idx.is_contiguous() or idx.device.type != "cuda":
        raise ValueError("idx must be a contiguous int32 device tensor")
    return ctypes.c_void_p(idx.data_ptr())


def _rp_ws(batch: int, workspace: Optional[torch.Tensor], dev) -> torch.Tensor:
    need = int(lib().hatt_rankpred_ws_bytes(int(batch)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    return workspace


def rankpred_grad(theta, stats, feat, label, idx, workspace=None, stream=None):
    """(gradient [NTHETA], loss [1]) of the mean loss over the rows idx."""
    B = idx.numel()
    grad = torch.empty(_lib.RANKPRED_NTHETA, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    ws = _rp_ws(B, workspace, feat.device)
    rows = feat.shape[0]
    check("hatt_rankpred_grad", lib().hatt_rankpred_grad(
        _f32(theta, "theta", _lib.RANKPRED_NTHETA), _f32(stats, "stats", _lib.RANKPRED_NSTATS),
        _f32(feat, "feat", rows * 21), _f32(label, "label", rows * 2), _idx(idx), B, _f32(grad, "grad"),
        _f32(loss, "loss"), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return grad, loss


def rankpred_train_step(theta, m, v, step: int, stats, feat, label, idx, *, lr: float = 1e-3,
                        beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, loss=None,
                        workspace=None, stream=None):
    """One Adam step in place on theta (m, v: its moments); returns the
    minibatch loss (device [1]) before the step."""
    B = idx.numel()
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    ws = _rp_ws(B, workspace, feat.device)
    rows = feat.shape[0]
    o = HattAdamOpts(float(lr), float(beta1), float(beta2), float(eps))
    n = _lib.RANKPRED_NTHETA
    check("hatt_rankpred_train_step", lib().hatt_rankpred_train_step(
        _f32(theta, "theta", n), _f32(m, "m", n), _f32(v, "v", n), int(step), ctypes.byref(o),
        _f32(stats, "stats", _lib.RANKPRED_NSTATS), _f32(feat, "feat", rows * 21), _f32(label, "label", rows * 2),
        _idx(idx), B, _f32(loss, "loss"), ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))
    return loss


def rankpred_widths(pairs, pred, margin: float = 0.0, oversample: int = 8):
    """Host: per pair (widths [d+1], predicted kept ranks [d+1]) from the
    predictions (host float32 array or device tensor [rows, 2])."""
    if isinstance(pred, torch.Tensor):
        pred = pred.detach().float().cpu().numpy()
    pred = np.ascontiguousarray(pred, dtype=np.float32)
    rows = rankpred_rows(pairs)
    if pred.shape != (rows, 2):
        raise ValueError(f"pred must be [{rows}, 2]")
    keep, xs, ys = _pair_views(pairs)
    ne = sum(x.d + 1 for x, _ in pairs)
    ell = (ctypes.c_int64 * ne)()
    rho = (ctypes.c_int64 * ne)()
    check("hatt_rankpred_widths", lib().hatt_rankpred_widths(
        len(pairs), xs, ys, ctypes.c_void_p(pred.ctypes.data), float(margin), int(oversample), ell, rho))
    out, e = [], 0
    for x, _ in pairs:
        out.append((list(ell[e:e + x.d + 1]), list(rho[e:e + x.d + 1])))
        e += x.d + 1
    return out


def adaptive_caps(x: TT, y: TT) -> List[int]:
    """Largest widths the tolerance mode may use for a pair: the feasible
    widths (the clamp of r_k s_k) limited to the 3072-column truncation."""
    xv, kx = x.view()
    yv, ky = y.view()
    o = HattAdaptOpts(1.0, 0, 8, 1, 1, 0.0, None, 0)
    cap = (ctypes.c_int64 * (x.d + 1))()
    ws = ctypes.c_size_t(0)
    oe = ctypes.c_int64(0)
    check("hatt_adaptive_plan", lib().hatt_adaptive_plan(ctypes.byref(xv), ctypes.byref(yv), ctypes.byref(o),
                                                         cap, ctypes.byref(ws), ctypes.byref(oe)))
    return list(cap)


def rankpred_labels(kept: Sequence[int], cap: Sequence[int], oversample: int = 8) -> np.ndarray:
    """Targets of the width predictor for one accepted recompression: per
    bond (ln rho_k, ln min(cap_k, rho_k + p))."""
    d = len(kept) - 1
    out = np.zeros((max(d - 1, 0), 2), dtype=np.float32)
    check("hatt_rankpred_labels", lib().hatt_rankpred_labels(d, i64_array(kept), i64_array(cap), int(oversample),
                                                             out.ctypes.data_as(ctypes.c_void_p)))
    return out


def kept_cores(res: Result, b: int = 0) -> List[torch.Tensor]:
    """Device cores of train b of a result, cut to its kept ranks."""
    kept = [int(v) for v in res.ranks[b].tolist()]
    return [res.out.core(k, b)[:kept[k], :, :kept[k + 1]] for k in range(res.out.d)]


def rel_err(a: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> float:
    """||a - b||_F / ||b||_F of two TTs given as device core lists (the error
    measure of Sec. 5), through the difference TT [a | -b] (interior cores
    block-diagonal, ranks r_a + r_b) and tt_norm."""
    d = len(a)
    n = [int(c.shape[1]) for c in a]
    ra = [1] + [int(c.shape[2]) for c in a]
    rb = [1] + [int(c.shape[2]) for c in b]
    flat = []
    for k in range(d):
        A, B = a[k], b[k]
        if d == 1:
            c = A - B
        elif k == 0:
            c = torch.cat([A, -B], dim=2)
        elif k == d - 1:
            c = torch.cat([A, B], dim=0)
        else:
            c = torch.zeros((ra[k] + rb[k], n[k], ra[k + 1] + rb[k + 1]), dtype=torch.float64, device=A.device)
            c[:ra[k], :, :ra[k + 1]] = A
            c[ra[k]:, :, ra[k + 1]:] = B
        flat.append(c.reshape(-1))
    ranks = [1] + [ra[k] + rb[k] for k in range(1, d)] + [1] if d > 1 else [1, 1]
    diff = TT(torch.cat(flat), n, ranks)
    base = TT(torch.cat([c.reshape(-1) for c in b]), n, rb)
    return float(norm(diff)[0].item() / norm(base)[0].item())
