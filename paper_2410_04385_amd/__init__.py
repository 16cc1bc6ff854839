"""MI355X-native HaTT: recompression of the Hadamard product of two tensor
trains without forming its partial Kronecker product cores.

The arithmetic lives in the HIP library ``libhatt.so`` (C ABI in
``include/hatt.h``); this package only marshals arguments and uses PyTorch
for device memory and streams.  Importing the package does not load the
library; the first call does, and fails loudly if it has not been built.
"""

from .api import (  # noqa: F401
    TT,
    Result,
    adaptive_caps,
    kept_cores,
    rankpred_labels,
    rel_err,
    batched_plan,
    batched_adaptive_plan,
    hadamard_explicit,
    hadamard_norm2,
    norm,
    plan,
    profile_report,
    profile_start,
    profile_stop,
    rankpred_features,
    rankpred_fit_stats,
    rankpred_forward,
    rankpred_grad,
    rankpred_rows,
    rankpred_train_step,
    rankpred_widths,
    recompress,
    recompress_adaptive,
    plan3,
    recompress3,
    recompress3_adaptive,
    recompress_batched,
    recompress_batched_adaptive,
    recompress_noalloc,
    randorth,
    round,
    round_plan,
    scale,
    check_finite,
    set_qr_method,
    sketch_fill,
    tune,
    tune_clear,
    tune_table,
    version,
)
from ._lib import HattError  # noqa: F401,E402
