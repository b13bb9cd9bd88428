"""Error metrics -- CPU ORACLE, test infrastructure.

Compression error of a decoded matrix against its uncompressed source, with
the conventions of the paper's Table 2 (Sec. 4.3): RMSE, NRMSE = RMSE /
(max - min) of the source, maximum pointwise error, PSNR = -20 log10(2 NRMSE)
(equivalently 20 log10(range / (2 RMSE))), and the compression ratio
32 / bits-per-value for FP32 data.  GEMV error: relative L2 against an FP64
reference, and the paper's quantity-of-interest check (relative error of
the product computed from the decoded matrix against the product from the
source matrix; the paper accepts below 1 %, Sec. 4.3).

Sums are FP64 (numpy, pairwise).  Only the test suite may import this.
"""
from __future__ import annotations

import math

import numpy as np


def compression_ratio(bits_per_value: float, value_bits: int = 32) -> float:
    return value_bits / bits_per_value


def rmse(src: np.ndarray, dec: np.ndarray) -> float:
    d = np.asarray(dec, dtype=np.float64) - np.asarray(src, dtype=np.float64)
    return float(np.sqrt(np.mean(d * d)))


def nrmse(src: np.ndarray, dec: np.ndarray) -> float:
    s = np.asarray(src, dtype=np.float64)
    return rmse(src, dec) / float(s.max() - s.min())


def max_pointwise_error(src: np.ndarray, dec: np.ndarray) -> float:
    return float(np.max(np.abs(np.asarray(dec, dtype=np.float64) - np.asarray(src, dtype=np.float64))))


def psnr_from_nrmse(nr: float) -> float:
    return -20.0 * math.log10(2.0 * nr)


def psnr(src: np.ndarray, dec: np.ndarray) -> float:
    return psnr_from_nrmse(nrmse(src, dec))


def rel_l2(y: np.ndarray, ref: np.ndarray) -> float:
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def gemv_flops(rows: int, cols: int, k: int = 1) -> int:
    """M(2N - 1) FLOP per product (Sec. 2.1, FLOP cost of a dense GEMV)."""
    return k * rows * (2 * cols - 1)


def gemv_ios(rows: int, cols: int) -> int:
    """MN + N + M values moved per product (Sec. 2.1, Eq. 4's GEMV term)."""
    return rows * cols + cols + rows


def pipeline_period(t_transfer: float, t_compute: float, t_decode: float = 0.0, ratio: float | None = None) -> float:
    """Table 1: max(T_transfer, T_compute) without compression,
    max(T_transfer / R, T_compute + T_decode) with it."""
    if ratio is None:
        return max(t_transfer, t_compute)
    return max(t_transfer / ratio, t_compute + t_decode)


def pipeline_latency(t_transfer: float, t_compute: float, t_decode: float = 0.0, ratio: float | None = None) -> float:
    """Table 1: T_compute + T_transfer, or T_compute + T_transfer / R + T_decode."""
    if ratio is None:
        return t_compute + t_transfer
    return t_compute + t_transfer / ratio + t_decode
