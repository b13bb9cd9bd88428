"""Pure-Python twin of the WHZ1 block codec -- CPU ORACLE, test infrastructure.

An independent second reading of the zfp-style fixed-rate code (the paper's
choice of zfp in fixed-rate mode, Sec. 4.3 "Data Compression", Table 2),
written in a different style from the C oracle (bit lists and Python
integers instead of byte buffers and machine words) so that the two can be
compared bit for bit on tiny inputs and on arbitrary byte strings.  Only for
small cases: every bit is a Python object.

Only the test suite may import this module.
"""
from __future__ import annotations

import math

import numpy as np

MASK32 = (1 << 32) - 1
NEGA = 0xAAAAAAAA


def wrap32(v: int) -> int:
    """Two's-complement int32 value of v modulo 2^32."""
    v &= MASK32
    return v - (1 << 32) if v >= (1 << 31) else v


def sequency_order() -> list[int]:
    """Local indices v = 4r + c sorted by (c + r, c^2 + r^2, larger c first)."""
    return sorted(range(16), key=lambda v: ((v & 3) + (v >> 2), (v & 3) ** 2 + (v >> 2) ** 2, -(v & 3)))


def lift(x: int, y: int, z: int, w: int) -> tuple[int, int, int, int]:
    """Forward decorrelating lift on four int32 values (floor halving)."""
    x = wrap32(x + w) >> 1
    w = wrap32(w - x)
    z = wrap32(z + y) >> 1
    y = wrap32(y - z)
    x = wrap32(x + z) >> 1
    z = wrap32(z - x)
    w = wrap32(w + y) >> 1
    y = wrap32(y - w)
    w = wrap32(w + (y >> 1))
    y = wrap32(y - (w >> 1))
    return x, y, z, w


def unlift(x: int, y: int, z: int, w: int) -> tuple[int, int, int, int]:
    """Inverse of `lift`: its five steps undone last-first."""
    y = wrap32(y + (w >> 1))
    w = wrap32(w - (y >> 1))
    y = wrap32(y + w)
    w = wrap32(2 * w - y)
    z = wrap32(z + x)
    x = wrap32(2 * x - z)
    y = wrap32(y + z)
    z = wrap32(2 * z - y)
    w = wrap32(w + x)
    x = wrap32(2 * x - w)
    return x, y, z, w


def forward_transform(block: list[int]) -> list[int]:
    """Lift every block row (over c), then every block column (over r)."""
    b = list(block)
    for r in range(4):
        b[4 * r:4 * r + 4] = lift(*b[4 * r:4 * r + 4])
    for c in range(4):
        col = lift(b[c], b[c + 4], b[c + 8], b[c + 12])
        for r in range(4):
            b[c + 4 * r] = col[r]
    return b


def inverse_transform(block: list[int]) -> list[int]:
    """Undo `forward_transform`: columns first, then rows."""
    b = list(block)
    for c in range(4):
        col = unlift(b[c], b[c + 4], b[c + 8], b[c + 12])
        for r in range(4):
            b[c + 4 * r] = col[r]
    for r in range(4):
        b[4 * r:4 * r + 4] = unlift(*b[4 * r:4 * r + 4])
    return b


def negabinary(i: int) -> int:
    return ((i + NEGA) & MASK32) ^ NEGA


def from_negabinary(n: int) -> int:
    return wrap32((n ^ NEGA) - NEGA)


def code_planes(coeffs: list[int], budget: int) -> list[int]:
    """Embedded group-testing code of 16 unsigned 32-bit coefficients,
    most significant plane first, truncated to `budget` bits."""
    out: list[int] = []
    sig = 0
    for p in range(31, -1, -1):
        if len(out) >= budget:
            break
        plane = [(c >> p) & 1 for c in coeffs]
        for s in range(sig):  # verbatim bits of significant coefficients
            if len(out) >= budget:
                break
            out.append(plane[s])
        # group tests over the remaining (insignificant) coefficients
        pos = sig
        while sig < 16 and len(out) < budget:
            rest = plane[pos:]
            if not any(rest):
                out.append(0)
                break
            out.append(1)
            while sig < 15 and len(out) < budget:
                out.append(plane[pos])
                if plane[pos]:
                    break
                pos += 1
                sig += 1
            pos += 1
            sig += 1
    return out[:budget]


def decode_planes(bits: list[int], budget: int) -> list[int]:
    """Inverse of `code_planes`; reads at most `budget` bits of `bits`."""
    it = iter(bits[:budget])
    used = 0
    coeffs = [0] * 16
    sig = 0

    def take() -> int:
        nonlocal used
        used += 1
        return next(it)

    for p in range(31, -1, -1):
        if used >= budget:
            break
        plane = [0] * 16
        for s in range(min(sig, budget - used)):
            plane[s] = take()
        while sig < 16 and used < budget:
            if not take():
                break
            while sig < 15 and used < budget:
                if take():
                    break
                sig += 1
            plane[sig] = 1
            sig += 1
        for s in range(16):
            coeffs[s] |= plane[s] << p
    return coeffs


def encode_block(f16, rate: int) -> list[int]:
    """Bits of one block (values in local order 4r + c), length 16*rate."""
    maxbits = 16 * rate
    vals = [float(np.float32(v)) for v in f16]
    if any(math.isnan(v) or math.isinf(v) for v in vals):
        raise ValueError("NaN/Inf cannot be encoded")
    nz = [v for v in vals if v != 0.0]
    if not nz:
        return [0] * maxbits
    emax = max(max(math.frexp(v)[1] for v in nz), -126)
    bits = [1] + [((emax + 127) >> k) & 1 for k in range(8)]
    ints = [int(math.ldexp(v, 30 - emax)) for v in vals]  # int() truncates toward zero
    coeffs = forward_transform(ints)
    order = sequency_order()
    nega = [negabinary(coeffs[order[s]]) for s in range(16)]
    bits += code_planes(nega, maxbits - 9)
    return bits + [0] * (maxbits - len(bits))


def decode_block(bits: list[int], rate: int) -> np.ndarray:
    """Values (float32, local order 4r + c) of one block's 16*rate bits."""
    maxbits = 16 * rate
    if not bits[0]:
        return np.zeros(16, dtype=np.float32)
    emax = sum(bits[1 + k] << k for k in range(8)) - 127
    nega = decode_planes(bits[9:maxbits], maxbits - 9)
    order = sequency_order()
    coeffs = [0] * 16
    for s in range(16):
        coeffs[order[s]] = from_negabinary(nega[s])
    ints = inverse_transform(coeffs)
    out = np.empty(16, dtype=np.float32)
    with np.errstate(over="ignore"):  # arbitrary bits may overflow to +-Inf, as IEEE rounding says
        for v in range(16):
            out[v] = np.float32(float(np.float32(ints[v])) * 2.0 ** (emax - 30))
    return out


def bytes_to_bits(data: bytes) -> list[int]:
    return [(byte >> k) & 1 for byte in data for k in range(8)]


def bits_to_bytes(bits: list[int]) -> bytes:
    assert len(bits) % 8 == 0
    return bytes(sum(bits[8 * i + k] << k for k in range(8)) for i in range(len(bits) // 8))


def encode_matrix(M: np.ndarray, rate: int) -> bytes:
    rows, cols = M.shape
    assert rows % 4 == 0 and cols % 4 == 0
    bits: list[int] = []
    for bi in range(rows // 4):
        for bj in range(cols // 4):
            blk = M[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4].reshape(16)
            bits += encode_block(blk, rate)
    return bits_to_bytes(bits)


def decode_matrix(stream: bytes, rows: int, cols: int, rate: int) -> np.ndarray:
    maxbits = 16 * rate
    bits = bytes_to_bits(stream)
    out = np.empty((rows, cols), dtype=np.float32)
    b = 0
    for bi in range(rows // 4):
        for bj in range(cols // 4):
            blk = decode_block(bits[b * maxbits:(b + 1) * maxbits], rate)
            out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4] = blk.reshape(4, 4)
            b += 1
    return out


def gemv_exact(Mhat: np.ndarray, u: np.ndarray) -> list[float]:
    """Correctly rounded y[i] = sum_j Mhat[i,j] * u[j] (math.fsum of the
    products, each exact in double since both factors are FP32)."""
    return [math.fsum(float(a) * float(b) for a, b in zip(row, u)) for row in Mhat]
