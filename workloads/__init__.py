"""Seeded synthetic inputs for the Hadamard-product recompression workloads.

This module is shared by the oracle, the tests and the benchmark.  It only
*draws* inputs (TT cores of the two factors, explicit Gaussian sketch cores
when a caller wants to pass the sketch in); it contains none of the
recompression arithmetic itself.

A TT tensor is a plain ``list`` of ``numpy.float64`` arrays; core ``k`` has
shape ``(rank[k], n[k], rank[k+1])`` with ``rank[0] == rank[d] == 1``.
The mode index is the middle axis and the multi-index is row-major
(last index fastest), the paper's convention of Sec. 2.1.
"""

from .gen import (  # noqa: F401
    WORKLOADS,
    gaussian_tt,
    spectral_tt,
    gaussian_sketch,
    trig_u,
    tiny_pair,
    spectral_pair,
    batched_pair_shapes,
    ranks_of,
    modes_of,
    feasible_ranks,
    mlp_init,
    separable_sum_tt,
    qing_values,
    alpine_values,
    qtt_sine,
    qtt_trig_field,
)
