"""Reference quantisers for reduced-precision matrix storage -- CPU ORACLE,
test infrastructure only.

The paper stores every real value as FP32 (Sec. 2.1) and multiplies in FP32
(Sec. 4.4).  The precision sweep stores the same matrix in narrower formats;
each is defined here from its number format, independently of the GPU code:

  FP16   IEEE binary16, round to nearest even from FP32 (numpy's cast)
  BF16   the top 16 bits of FP32 after round to nearest even
  FP8    OCP e4m3 (bias 7, 3 mantissa bits, max 448, no infinities) with one
         FP32 scale per 4x4 block: s = amax / 448, code = RNE_sat(f * (448 /
         amax)) with both FP32 operations correctly rounded; value = e4m3(code)
         * s.  A zero block has s = 0 and all codes 0.
"""
from __future__ import annotations

import numpy as np


def to_f16(M: np.ndarray) -> np.ndarray:
    return np.asarray(M, dtype=np.float32).astype(np.float16)


def bf16_bits(M: np.ndarray) -> np.ndarray:
    """uint16 BF16 codes, round to nearest even (finite inputs)."""
    b = np.ascontiguousarray(M, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_values(codes: np.ndarray) -> np.ndarray:
    return (codes.astype(np.uint32) << 16).view(np.float32)


def e4m3_value(code: int) -> float:
    """Value of an OCP e4m3 code (NaN for S.1111.111)."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 7
    if e == 15 and m == 7:
        return float("nan")
    if e == 0:
        return s * m * 2.0 ** -9
    return s * (1.0 + m / 8.0) * 2.0 ** (e - 7)


E4M3_TABLE = np.array([e4m3_value(c) for c in range(256)], dtype=np.float64)
_POS = np.array([E4M3_TABLE[c] for c in range(0x7F)], dtype=np.float64)  # codes 0..126, ascending


def e4m3_rne_sat(x: np.ndarray) -> np.ndarray:
    """Nearest e4m3 code (ties to even code), saturating at +-448."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    idx = np.searchsorted(_POS, a)           # first code with value >= a
    hi = np.minimum(idx, 0x7E)
    lo = np.maximum(hi - 1, 0)
    dlo = a - _POS[lo]
    dhi = _POS[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    code = np.where(a == _POS[hi], hi, code).astype(np.uint8)
    sign = (np.signbit(x) & (code != 0)).astype(np.uint8) << 7
    return (code | sign).astype(np.uint8)


def fp8_block_scaled(M: np.ndarray):
    """(codes (nb, 16) uint8 in block order, scales (nb,) float32)."""
    M = np.asarray(M, dtype=np.float32)
    R, C = M.shape
    blocks = M.reshape(R // 4, 4, C // 4, 4).transpose(0, 2, 1, 3).reshape(-1, 16)
    amax = np.abs(blocks).max(axis=1).astype(np.float32)
    nz = amax > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(nz, amax / np.float32(448.0), np.float32(0.0)).astype(np.float32)
        inv = np.where(nz, np.float32(448.0) / amax, np.float32(0.0)).astype(np.float32)
    scaled = (blocks * inv[:, None]).astype(np.float32)   # one FP32 rounding
    codes = e4m3_rne_sat(scaled)
    codes[~nz] = 0
    return codes, s


def fp8_dequant(codes: np.ndarray, scales: np.ndarray, R: int, C: int) -> np.ndarray:
    """The dequantised matrix in FP64 (exact products of e4m3 values and FP32 scales)."""
    vals = E4M3_TABLE[codes] * scales.astype(np.float64)[:, None]
    return vals.reshape(R // 4, C // 4, 4, 4).transpose(0, 2, 1, 3).reshape(R, C)
