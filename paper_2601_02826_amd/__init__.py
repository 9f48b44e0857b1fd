"""MI355X-native FS-QRPPA: weighted-l1 penalized quantile regression on gfx950.

The solver lives in libpqr.so (hand-written HIP kernels behind the C ABI of
include/pqr.h); this package is its thin Python binding.
"""
from ._lib import (Context, PQRError, Result, load, LIB_PATH, SYMBOLS, FMT, START,  # noqa: F401
                   PQR_OK, PQR_ERR_INVALID_ARG, PQR_ERR_OOM, PQR_ERR_DEVICE,
                   PQR_ERR_NOT_CONVERGED, PQR_ERR_DIVERGED, PQR_ERR_UNSUPPORTED,
                   mlp_param_count, mlp_forward, mlp_workspace_bytes, mlp_grad, mlp_grad_noalloc, MLP_NOALLOC_MAX_ROWS, mlp_adam,
                   solve_grouped, interleaved_order, Interleaved, TILE_VARIANTS, BGEMM_VARIANTS,
                   BAXPY_VARIANTS)

create = Context
