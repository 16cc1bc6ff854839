"""FP64 CPU oracle for Hadamard-avoiding TT recompression (HaTT).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library.

Everything here is plain, slow and written to be read against the paper
("HaTT: Hadamard avoiding TT recompression and its applications"):

* ``tt``        TT containers, the full tensor, the partial Kronecker product
                (PKP) cores of a Hadamard product (Sec. 2.2), Frobenius norm and
                the relative error of Sec. 5 computed through a difference TT.
* ``rounding``  TT-Rounding (Alg. 1) with a rank cap and/or a tolerance.
* ``randorth``  PartialContractionRL (eq. rtlpc) and RandOrth (Alg. 2).
* ``hatt``      HPCRL (Alg. 3; HaTT-1 and HaTT-2 splits, eqs. HPCRL--1/--2)
                and HaTT (Alg. 4) without forming PKP cores.
* ``hatt3``     the same for three factors, x (.) y (.) w, by three-mode
                products (the Kronecker-times-vector identity taken over three
                factors; an extension the paper does not spell out).
* ``plan``      the sketch-width clamps applied before a recompression.
* ``philox``    the counter-based generator of the seeded Gaussian sketch.
* ``flops``     the paper's operation counts (Sec. 4, Table 4.1).
* ``adapt``     tolerance-driven widths (grow l until the truncation leaves
                slack; Sec. 5.1.1 and Sec. 6 leave the rule open).
* ``rankpred``  the per-bond width predictor: core statistics, a small tanh
                MLP, its gradient and the Adam update.
* ``power``     the power iteration for a TT's largest entry with HaTT
                recompressions (Sec. 5, Example 3).

All arithmetic is numpy float64; QR and SVD are LAPACK calls (Householder QR
and divide-and-conquer SVD), used only as library steps.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
(brute force on full tensors, closed forms, invariants and theorem
inequalities); none is "parity unpinned".
"""

from . import tt, rounding, randorth, hatt, hatt3, plan, philox, flops, adapt, rankpred, power  # noqa: F401
