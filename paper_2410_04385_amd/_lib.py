"""ctypes declarations of the C ABI in include/hatt.h (argument marshalling
only).  Loading fails loudly when libhatt.so has not been built: there is no
fallback implementation."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhatt.so")

HATT_OK = 0
STATUS_NAMES = {
    0: "HATT_OK", -1: "HATT_EINVAL", -2: "HATT_ESHAPE", -3: "HATT_EWORKSPACE", -4: "HATT_EDEVICE",
    -5: "HATT_ENOTCONV", -6: "HATT_ENONFINITE", -7: "HATT_EUNSUPPORTED",
}

EXPORTED = [
    "hatt_plan", "hatt_recompress", "hatt_recompress_noalloc", "hatt_adaptive_plan", "hatt_recompress_adaptive", "tt_hadamard_explicit", "tt_scale", "tt_check_finite", "tt_randorth_plan", "tt_randorth", "tt_round_plan", "tt_round",
    "tt_norm_plan", "tt_norm", "hatt_sketch_fill", "hatt_profile_start", "hatt_profile_stop",
    "hatt_profile_class_name", "hatt_last_error", "hatt_version", "hatt_set_qr_method",
    "hatt_profile_report", "hatt_batched_plan", "hatt_recompress_batched",
    "hatt_rankpred_features", "hatt_rankpred_fit_stats", "hatt_rankpred_forward", "hatt_rankpred_ws_bytes",
    "hatt_rankpred_grad", "hatt_rankpred_train_step", "hatt_rankpred_widths", "hatt_rankpred_labels",
    "hatt_plan3", "hatt_recompress3", "hatt_adaptive_plan3", "hatt_recompress3_adaptive",
    "hatt_tune_mode", "hatt_tune_clear", "hatt_tune_table", "hatt_hadamard_norm2_plan", "hatt_hadamard_norm2",
    "hatt_batched_adaptive_plan", "hatt_recompress_batched_adaptive",
]
RANKPRED_NIN, RANKPRED_NTHETA, RANKPRED_NSTATS = 21, 19586, 46
PROFILE_CLASSES = 8

i64p = ctypes.POINTER(ctypes.c_int64)


class HattTT(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("n", i64p),
        ("rank", i64p),
        ("data", ctypes.c_void_p),
        ("batch_stride", ctypes.c_int64),
    ]


class HattOpts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("ep", ctypes.c_double),
        ("ell", ctypes.c_int64),
        ("ell_bond", i64p),
        ("max_rank", ctypes.c_int64),
        ("tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int32),
        ("max_rank_bond", i64p),
    ]


class HattAdaptOpts(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("oversample", ctypes.c_int32),
        ("max_attempts", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("ep", ctypes.c_double),
        ("ell_init", i64p),
        ("precision", ctypes.c_int32),
    ]


class HattAdamOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class HattError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2410_04385_amd.build` "
            "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, ttp, optp = ctypes.c_void_p, ctypes.POINTER(HattTT), ctypes.POINTER(HattOpts)
    szp = ctypes.POINTER(ctypes.c_size_t)
    L.hatt_plan.argtypes = [ttp, ttp, optp, i64p, szp, i64p]
    L.hatt_recompress.argtypes = [ttp, ttp, ttp, optp, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
    L.hatt_recompress_noalloc.argtypes = [ttp, ttp, ttp, optp, vp, ctypes.c_int64, vp, vp]
    aop = ctypes.POINTER(HattAdaptOpts)
    L.hatt_adaptive_plan.argtypes = [ttp, ttp, aop, i64p, szp, i64p]
    L.hatt_recompress_adaptive.argtypes = [ttp, ttp, aop, vp, ctypes.c_int64, vp, i64p,
                                           ctypes.POINTER(ctypes.c_int32), vp, ctypes.c_size_t, vp]
    L.hatt_batched_adaptive_plan.argtypes = [ctypes.c_int32, ttp, ttp, aop, i64p, i64p, i64p, szp, szp]
    L.hatt_recompress_batched_adaptive.argtypes = [ctypes.c_int32, ttp, ttp, aop, vp, vp, i64p,
                                                   ctypes.POINTER(ctypes.c_int32), vp, ctypes.c_size_t, vp]
    L.hatt_plan3.argtypes = [ttp, ttp, ttp, optp, i64p, szp, i64p]
    L.hatt_recompress3.argtypes = [ttp, ttp, ttp, ttp, optp, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
    L.hatt_adaptive_plan3.argtypes = [ttp, ttp, ttp, aop, i64p, szp, i64p]
    L.hatt_recompress3_adaptive.argtypes = [ttp, ttp, ttp, aop, vp, ctypes.c_int64, vp, i64p,
                                            ctypes.POINTER(ctypes.c_int32), vp, ctypes.c_size_t, vp]
    L.tt_hadamard_explicit.argtypes = [ttp, ttp, vp, ctypes.c_int64, vp]
    L.hatt_hadamard_norm2_plan.argtypes = [ttp, ttp, szp]
    L.hatt_hadamard_norm2.argtypes = [ttp, ttp, vp, vp, ctypes.c_size_t, vp]
    L.tt_randorth_plan.argtypes = [ttp, ctypes.c_int64, i64p, i64p, szp, i64p]
    L.tt_randorth.argtypes = [ttp, ttp, ctypes.c_int64, i64p, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, vp,
                              ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
    L.tt_scale.argtypes = [ttp, vp, ctypes.c_int32, vp]
    L.hatt_rankpred_labels.argtypes = [ctypes.c_int32, i64p, i64p, ctypes.c_int32, vp]
    L.tt_check_finite.argtypes = [ttp, vp, vp]
    L.tt_round_plan.argtypes = [ttp, i64p, szp, i64p]
    L.tt_round.argtypes = [ttp, ctypes.c_int64, ctypes.c_double, vp, ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
    L.tt_norm_plan.argtypes = [ttp, szp]
    L.tt_norm.argtypes = [ttp, vp, vp, ctypes.c_size_t, vp]
    L.hatt_sketch_fill.argtypes = [ctypes.c_uint64, ctypes.c_int32, i64p, i64p, vp, vp]
    i64, sz = ctypes.c_int64, ctypes.c_size_t
    L.hatt_rankpred_features.argtypes = [ctypes.c_int32, ttp, ttp, vp, vp]
    L.hatt_rankpred_fit_stats.argtypes = [vp, vp, i64, vp, vp]
    L.hatt_rankpred_forward.argtypes = [vp, vp, vp, i64, vp, vp]
    L.hatt_rankpred_ws_bytes.argtypes = [i64]
    L.hatt_rankpred_grad.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, sz, vp]
    L.hatt_rankpred_train_step.argtypes = [vp, vp, vp, i64, ctypes.POINTER(HattAdamOpts), vp, vp, vp, vp, i64, vp,
                                           vp, sz, vp]
    L.hatt_rankpred_widths.argtypes = [ctypes.c_int32, ttp, ttp, vp, ctypes.c_double, ctypes.c_int32, i64p, i64p]
    L.hatt_profile_start.argtypes = []
    L.hatt_profile_stop.argtypes = [ctypes.POINTER(ctypes.c_double), i64p]
    L.hatt_profile_class_name.argtypes = [ctypes.c_int32]
    L.hatt_profile_class_name.restype = ctypes.c_char_p
    for fn in EXPORTED:
        if fn not in ("hatt_profile_class_name", "hatt_last_error", "hatt_version", "hatt_profile_report",
                      "hatt_rankpred_ws_bytes", "hatt_tune_table"):
            getattr(L, fn).restype = ctypes.c_int
    L.hatt_last_error.restype = ctypes.c_char_p
    L.hatt_version.restype = ctypes.c_char_p
    L.hatt_profile_report.restype = ctypes.c_char_p
    L.hatt_rankpred_ws_bytes.restype = ctypes.c_size_t
    L.hatt_tune_table.restype = ctypes.c_int64
    L.hatt_tune_table.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    L.hatt_tune_mode.argtypes = [ctypes.c_int32]
    _lib = L
    return L


def check(fn: str, status: int) -> None:
    if status != HATT_OK:
        msg = lib().hatt_last_error().decode(errors="replace")
        raise HattError(fn, status, msg)


def i64_array(values):
    arr = (ctypes.c_int64 * len(values))(*[int(v) for v in values])
    return arr
