"""Algorithmic operation counts of the kernels the library launches for one
HaTT-1 recompression followed by TT-Rounding, per kernel class.

Counts follow the complexity paragraphs of Sec. 4 term by term, with the
actual per-bond ranks: x ranks r_k, y ranks s_k, sketch widths l_k (also the
ranks entering the rounding), output caps c_k.  Flops of the iterative
Jacobi SVD are not counted (they depend on the number of sweeps).
"""

from __future__ import annotations

from typing import Dict, Sequence

# MI355X published peaks used as roofline denominators
PEAK_FP64_TFLOPS = 78.6      # FP64 vector and FP64 matrix cores alike
PEAK_FP32_TFLOPS = 157.3     # FP32 (dense, matrix cores)
PEAK_BF16_TFLOPS = 2500.0    # BF16 (dense, matrix cores)


def mfma_peak_tflops(kernel: str) -> float:
    """Dense matrix-core peak of the type a kernel computes in, read off its
    name (the FP32 and BF16 range-finding instantiations name their type)."""
    if "bf16" in kernel:
        return PEAK_BF16_TFLOPS
    if "f32" in kernel or "float" in kernel:
        return PEAK_FP32_TFLOPS
    return PEAK_FP64_TFLOPS
PEAK_HBM_GBS = 8000.0


def _qr_flops(m: int, n: int) -> float:
    """Economy Householder QR forming Q (Sec. 4): 4 m n^2 - 4 n^3 / 3.  This
    algorithmic count is kept whatever QR method runs (CholeskyQR2 performs
    about 8 m n^2)."""
    k = min(m, n)
    return 4.0 * m * k * k - 4.0 * k ** 3 / 3.0


def hatt_round_flops(n: Sequence[int], r: Sequence[int], s: Sequence[int], ell: Sequence[int],
                     cap: int | None = None) -> Dict[str, float]:
    d = len(n)
    out = {"sandwich": 0.0, "gemm_f64": 0.0, "qr": 0.0}
    # HPCRL: W_L columns (Z U Y^T per (i, gamma)) and W_L W_R^T
    for c in range(1, d - 1):
        r0, r1, s0, s1, l0, l1 = r[c], r[c + 1], s[c], s[c + 1], ell[c], ell[c + 1]
        out["sandwich"] += 2.0 * n[c] * l1 * (r1 * s1 * s0 + r0 * r1 * s0)
        out["gemm_f64"] += 2.0 * (r0 * s0) * l0 * (n[c] * l1)
    # sweep: X W, QR, Q^T X, PKP-free update of the next core
    for c in range(d - 1):
        m = ell[c] * n[c]
        rs1 = r[c + 1] * s[c + 1]
        out["gemm_f64"] += 2.0 * m * ell[c + 1] * rs1 + 2.0 * ell[c + 1] * rs1 * m
        out["qr"] += _qr_flops(m, ell[c + 1])
        cn = c + 1
        out["sandwich"] += 2.0 * n[cn] * ell[cn] * (r[cn] * s[cn] * s[cn + 1] + r[cn + 1] * r[cn] * s[cn + 1])
    if cap is not None and d > 1:
        # truncation of the left-orthogonal rank-l result from the right (no
        # orthogonalisation pass): per bond the QR of the transposed
        # unfolding, the kept core (Q W) and the absorb of (U S) into the
        # core to its left
        caps = [1] + [min(cap, ell[k]) for k in range(1, d)] + [1]
        for c in range(d - 1, 0, -1):
            m = n[c] * caps[c + 1]
            out["qr"] += _qr_flops(m, ell[c])
            out["gemm_f64"] += 2.0 * m * ell[c] * caps[c]
            out["gemm_f64"] += 2.0 * ell[c - 1] * n[c - 1] * ell[c] * caps[c]
    out["total"] = sum(out.values())
    return out


def chatt_paper(d: int, n: int, r: int, s: int, ell: int) -> float:
    """eq. (CHATT) with HPCRL-1: (d-2) n r s l (4r + 4s + 6l)."""
    return (d - 2) * n * r * s * ell * (4 * r + 4 * s + 6 * ell)
