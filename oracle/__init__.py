"""FP64 CPU oracle for weighted-l1 penalized quantile regression (PQR) and FS-QRPPA.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the tests, the package's smoke
check and the CPU-baseline leg of the benchmark may import it.  The GPU
solver never calls into it and shares no code with it.

Contents (each function cites the passage of the paper it follows):

  pqr.py    objective, the two closed-form prox maps, Algorithm 1 step by step,
            lambda_max, the dual certificate, the KKT check, standardisation,
            the SCAD/MCP derivatives used by Algorithm 2
  lp.py     the l1-QR linear program solved exactly in rationals (Bland's-rule
            simplex), a brute-force vertex enumeration for tiny inputs, and a
            HiGHS cross-check
  mlp.py    the per-feature 4-64-64-2 scoring network, forward and backward in FP64

Parity status of every function is listed in the module docstrings; a function
with no independent pin says "parity unpinned".
"""
from . import pqr, lp, mlp  # noqa: F401
