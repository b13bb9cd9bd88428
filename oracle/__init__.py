"""CPU oracle for the compressed-matrix GEMV -- TEST INFRASTRUCTURE ONLY.

Only the test suite, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  It shares no code with the GPU library.

Contents:
  whz_oracle.c  scalar C: WHZ1 encode/decode (fixed rate, and the
                fixed-precision and fixed-accuracy modes with a block index),
                FP64 GEMV, the paper's mixed-precision GEMV (Fig. 7), dense
                references
  twin.py       pure-Python twin of the codec for tiny inputs
  metrics.py    compression-error and GEMV-error metrics (Table 2 conventions)
  quant.py      reference quantisers for the reduced-precision storage formats
  thermal.py    the thermal step of Eq. 1 (sparse A T + diagonal B u), FP64
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "whz_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, U32, U64, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.orc_encode.argtypes = [P, U32, U32, U32, P]
        L.orc_decode.argtypes = [P, U32, U32, U32, P]
        L.orc_decode_blocks.argtypes = [P, U32, U64, U64, P]
        L.orc_gemv_fp64.argtypes = [P, U32, U32, U32, P, U32, U32, P, I32]
        L.orc_gemv_paper_mp.argtypes = [P, U32, U32, U32, P, U32, U32, P, I32]
        L.orc_dense_gemv_fp64.argtypes = [P, U32, U32, P, P]
        L.orc_dense_gemv_paper_mp.argtypes = [P, U32, U32, P, P]
        L.orc_dense_gemv_fp32_naive.argtypes = [P, U32, U32, P, P]
        L.orc_var_groups.argtypes = [U32]
        L.orc_var_groups.restype = U32
        L.orc_var_capacity_bytes.argtypes = [U32, U32]
        L.orc_var_capacity_bytes.restype = U64
        L.orc_encode_var.argtypes = [P, U32, U32, I32, I32, P, U64, P, P]
        L.orc_decode_var.argtypes = [P, P, U32, U32, I32, I32, P]
        L.orc_encode_planes.argtypes = [P, ctypes.c_uint, P]
        L.orc_encode_planes.restype = ctypes.c_uint
        L.orc_decode_planes.argtypes = [P, ctypes.c_uint, P]
        L.orc_decode_planes.restype = ctypes.c_uint
        for name in ("orc_fwd_lift4", "orc_inv_lift4", "orc_fwd_xform", "orc_inv_xform", "orc_sequency_order"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


class OracleError(RuntimeError):
    pass


def _check(st: int) -> None:
    if st != 0:
        raise OracleError(f"oracle status {st}")


def stream_nbytes(rows: int, cols: int, rate: int) -> int:
    """Fixed rate: exactly 16*rate bits per 4x4 block; a dimension that is
    not a multiple of 4 ends in a partial (edge-padded) block."""
    return ((rows + 3) // 4) * ((cols + 3) // 4) * 2 * rate


def encode(M: np.ndarray, rate: int) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float32)
    rows, cols = M.shape
    out = np.zeros(stream_nbytes(rows, cols, rate), dtype=np.uint8)
    _check(lib().orc_encode(_ptr(M), rows, cols, rate, _ptr(out)))
    return out


def decode(stream: np.ndarray, rows: int, cols: int, rate: int) -> np.ndarray:
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    out = np.empty((rows, cols), dtype=np.float32)
    _check(lib().orc_decode(_ptr(stream), rows, cols, rate, _ptr(out)))
    return out


# ------------------------------------------------- variable-rate modes
VAR_PRECISION, VAR_ACCURACY = 0, 1
VAR_GROUP = 32  # block columns per index entry


def var_groups(cols: int) -> int:
    return int(lib().orc_var_groups(cols))


def encode_var(M: np.ndarray, mode: int, param: int):
    """Fixed-precision (mode 0, param = planes) or fixed-accuracy (mode 1,
    param = minexp: tolerance 2^minexp) code of M.  Returns (stream bytes,
    index uint64 [ceil(rows/4) * var_groups(cols)], bits)."""
    M = np.ascontiguousarray(M, dtype=np.float32)
    rows, cols = M.shape
    cap = int(lib().orc_var_capacity_bytes(rows, cols))
    out = np.zeros(cap, dtype=np.uint8)
    index = np.zeros(((rows + 3) // 4) * var_groups(cols), dtype=np.uint64)
    nbits = ctypes.c_uint64(0)
    _check(lib().orc_encode_var(_ptr(M), rows, cols, mode, param, _ptr(out), cap, _ptr(index), ctypes.byref(nbits)))
    return out[: (nbits.value + 7) // 8].copy(), index, nbits.value


def decode_var(stream: np.ndarray, index, rows: int, cols: int, mode: int, param: int) -> np.ndarray:
    """Decode with the index (index=None: blocks read one after another).
    `stream` may be the trimmed bytes: it is padded here for the reader."""
    buf = np.zeros(np.asarray(stream).size + 256, dtype=np.uint8)
    buf[: np.asarray(stream).size] = stream
    out = np.empty((rows, cols), dtype=np.float32)
    ip = None
    if index is not None:
        index = np.ascontiguousarray(index, dtype=np.uint64)
        ip = _ptr(index)
    _check(lib().orc_decode_var(_ptr(buf), ip, rows, cols, mode, param, _ptr(out)))
    return out


def decode_blocks(stream: np.ndarray, rate: int, b0: int, nblocks: int) -> np.ndarray:
    """Blocks [b0, b0+nblocks) as (nblocks, 16) float32, local order 4r + c."""
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    assert (b0 + nblocks) * 2 * rate <= stream.size
    out = np.empty((nblocks, 16), dtype=np.float32)
    _check(lib().orc_decode_blocks(_ptr(stream), rate, b0, nblocks, _ptr(out)))
    return out


def gemv_fp64(stream: np.ndarray, rows: int, cols: int, rate: int, u: np.ndarray,
              row_begin: int = 0, row_end: int | None = None, nthreads: int = 1) -> np.ndarray:
    """FP64 y over the oracle-decoded matrix for rows [row_begin, row_end)
    (any range inside the matrix); `stream` is the whole matrix's code."""
    row_end = rows if row_end is None else row_end
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    u = np.ascontiguousarray(u, dtype=np.float32)
    assert u.size == cols
    y = np.empty(max(row_end - row_begin, 0), dtype=np.float64)
    _check(lib().orc_gemv_fp64(_ptr(stream), rows, cols, rate, _ptr(u), row_begin, row_end, _ptr(y), nthreads))
    return y


def gemv_paper_mp(stream: np.ndarray, rows: int, cols: int, rate: int, u: np.ndarray,
                  row_begin: int = 0, row_end: int | None = None, nthreads: int = 1) -> np.ndarray:
    row_end = rows if row_end is None else row_end
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    u = np.ascontiguousarray(u, dtype=np.float32)
    y = np.empty(max(row_end - row_begin, 0), dtype=np.float32)
    _check(lib().orc_gemv_paper_mp(_ptr(stream), rows, cols, rate, _ptr(u), row_begin, row_end, _ptr(y), nthreads))
    return y


def dense_gemv_fp64(M: np.ndarray, u: np.ndarray) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32)
    y = np.empty(M.shape[0], dtype=np.float64)
    lib().orc_dense_gemv_fp64(_ptr(M), M.shape[0], M.shape[1], _ptr(u), _ptr(y))
    return y


def dense_gemv_paper_mp(M: np.ndarray, u: np.ndarray) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32)
    y = np.empty(M.shape[0], dtype=np.float32)
    lib().orc_dense_gemv_paper_mp(_ptr(M), M.shape[0], M.shape[1], _ptr(u), _ptr(y))
    return y


def dense_gemv_fp32_naive(M: np.ndarray, u: np.ndarray) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32)
    y = np.empty(M.shape[0], dtype=np.float32)
    lib().orc_dense_gemv_fp32_naive(_ptr(M), M.shape[0], M.shape[1], _ptr(u), _ptr(y))
    return y


def encode_planes(n16, budget: int) -> tuple[np.ndarray, int]:
    n16 = np.ascontiguousarray(n16, dtype=np.uint32)
    out = np.zeros((budget + 7) // 8 + 8, dtype=np.uint8)
    used = lib().orc_encode_planes(_ptr(n16), budget, _ptr(out))
    return out, int(used)


def decode_planes(buf: np.ndarray, budget: int) -> tuple[np.ndarray, int]:
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    assert buf.size * 8 >= budget
    n16 = np.zeros(16, dtype=np.uint32)
    used = lib().orc_decode_planes(_ptr(buf), budget, _ptr(n16))
    return n16, int(used)


def _int_op(name: str, v, n: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(v, dtype=np.int64).astype(np.int32))
    assert a.size == n
    getattr(lib(), name)(_ptr(a))
    return a


def fwd_lift4(v):
    return _int_op("orc_fwd_lift4", v, 4)


def inv_lift4(v):
    return _int_op("orc_inv_lift4", v, 4)


def fwd_xform(b16):
    return _int_op("orc_fwd_xform", b16, 16)


def inv_xform(b16):
    return _int_op("orc_inv_xform", b16, 16)


def sequency_order() -> list[int]:
    a = np.zeros(16, dtype=np.int32)
    lib().orc_sequency_order(_ptr(a))
    return [int(x) for x in a]
