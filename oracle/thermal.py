"""Oracle for the thermal step -- TEST INFRASTRUCTURE ONLY.

Eq. 1 of the paper (Sec. 2.1): T_{k+1} = A T_k + B u_k, A sparse (here in
CSR: row_ptr, col, val), B diagonal (its diagonal b).  Written as the
definition, in FP64: each row's products A_ij T_j summed in the order the row
lists them, plus b_i u_i.  The stored temperature state is FP32, so a run of
steps rounds each T_{k+1} once to FP32 before the next step.

Shares no code with the GPU library; only tests, smoke() and bench.py's CPU
baseline use it.
"""
from __future__ import annotations

import numpy as np


def thermal_step(row_ptr, col, val, b, T, u) -> np.ndarray:
    """FP64 T_{k+1} (not rounded)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    prod = np.asarray(val, dtype=np.float64) * np.asarray(T, dtype=np.float64)[np.asarray(col, dtype=np.int64)]
    y = np.bincount(rows, weights=prod, minlength=n)  # sequential FP64 sum, in entry order
    return y + np.asarray(b, dtype=np.float64) * np.asarray(u, dtype=np.float64)


def thermal_run(row_ptr, col, val, b, T0, U) -> np.ndarray:
    """T_K (FP32) after K = len(U) steps from T_0, u_k = U[k]."""
    T = np.asarray(T0, dtype=np.float32)
    for k in range(len(U)):
        T = thermal_step(row_ptr, col, val, b, T, U[k]).astype(np.float32)
    return T
