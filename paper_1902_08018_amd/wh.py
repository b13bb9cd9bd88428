"""Python binding of libwh (include/wh.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does
nothing but check Python-side types, pass raw pointers (torch tensors give
device memory, `torch.cuda.current_stream()` gives the stream) and turn a
non-OK status into `WhError`.  All the work runs in the HIP library; there is
no fallback: if libwh.so is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime that libwh.so shares  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwh.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libwh.so is not built ({LIB_PATH}); run __graft_entry__.build()")

_lib = ctypes.CDLL(LIB_PATH)

WH_OK, WH_PENDING = 0, 1
WH_ERR_INVALID, WH_ERR_SHAPE, WH_ERR_FORMAT, WH_ERR_NOMEM = -1, -2, -3, -4
WH_ERR_BUDGET, WH_ERR_DEVICE, WH_ERR_NOT_FOUND, WH_ERR_SCRATCH = -5, -6, -7, -8
WH_NOALLOC_SCRATCH_BYTES = 64 << 20

WH_FMT_ZFP_FIXED_RATE, WH_FMT_F32, WH_FMT_F16, WH_FMT_BF16, WH_FMT_FP8E4M3_BS4 = 1, 2, 3, 4, 5
WH_FMT_ZFP_FIXED_PRECISION, WH_FMT_ZFP_FIXED_ACCURACY = 6, 7


def accuracy_rate(minexp: int) -> int:
    """desc.rate of WH_FMT_ZFP_FIXED_ACCURACY for the tolerance 2^minexp."""
    return minexp + 1024
WH_HOST, WH_DEVICE = 0, 1
WH_ACC_DEFAULT, WH_ACC_FP64, WH_ACC_TWOSUM, WH_PAPER_MP, WH_HOST_DIRECT = 0, 1, 2, 4, 8
WH_U_F32, WH_U_BF16 = 0, 1


class WhError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {wh_status_str(status)} ({status})")


class wh_matrix_desc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint32), ("cols", ctypes.c_uint32), ("fmt", ctypes.c_int32),
                ("rate", ctypes.c_uint32)]


class wh_request(ctypes.Structure):
    _fields_ = [("mat", ctypes.c_uint64), ("U", ctypes.c_void_p), ("u_on_device", ctypes.c_int),
                ("k", ctypes.c_uint32), ("Y", ctypes.c_void_p), ("y_on_device", ctypes.c_int),
                ("deadline_ns", ctypes.c_uint64), ("arrival_ns", ctypes.c_uint64)]


class wh_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_arrive_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("missed", ctypes.c_int32), ("batch_size", ctypes.c_uint32)]


_P, _U32, _U64, _I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
_sig = {
    "wh_status_str": ([_I32], ctypes.c_char_p),
    "wh_create": ([ctypes.c_int, _U64, ctypes.POINTER(ctypes.c_void_p)], _I32),
    "wh_destroy": ([_P], _I32),
    "wh_storage_bytes": ([ctypes.POINTER(wh_matrix_desc), ctypes.POINTER(_U64)], _I32),
    "wh_load_compressed": ([_P, ctypes.POINTER(wh_matrix_desc), _P, _U64, ctypes.c_int, ctypes.POINTER(_U64)],
                           _I32),
    "wh_unload": ([_P, _U64], _I32),
    "wh_gemv": ([_P, _U64, _P, _P, _U32, _U32, _U32, _P], _I32),
    "wh_gemv_noalloc": ([_P, _U64, _P, _P, _U32, _U32, _U32, _P], _I32),
    "wh_gemv_batched": ([_P, _U64, _P, ctypes.c_int, _U32, _U32, _P, _U32, _U32, _P], _I32),
    "wh_gemv_host": ([_P, _P, _U32, _U32, _U32, _P, _P, _U32, _U32, _U32, _U32, _P], _I32),
    "wh_gemv_plan_info": ([_U32, _U32, _U32, _U32, ctypes.c_int, _U32, ctypes.POINTER(_U32)], _I32),
    "wh_var_index_bytes": ([_U32, _U32], _U64),
    "wh_var_capacity_bytes": ([_U32, _U32], _U64),
    "wh_encode_var": ([_P, _U32, _U32, _I32, _U32, _P, _U64, ctypes.POINTER(_U64)], _I32),
    "wh_host_alloc": ([_U64, ctypes.POINTER(ctypes.c_void_p)], _I32),
    "wh_host_free": ([_P], _I32),
    "wh_thermal_step": ([_P, _U32, _U32, _P, _P, _P, _P, _P, _P, _P, _P], _I32),
    "wh_thermal_run": ([_P, _U32, _U32, _P, _P, _P, _P, _P, _P, _U64, _U32, _P, _P], _I32),
    "wh_decode_debug": ([_P, _U64, _U64, _U64, _P, _P], _I32),
    "wh_decode": ([_P, _U64, _P, _P], _I32),
    "wh_encode": ([_P, _P, _U32, _U32, _U32, _P, _P, _P], _I32),
    "wh_quantize": ([_P, _P, _U32, _U32, _I32, _P, _P], _I32),
    "wh_stream_read": ([_P, _P, _U64, _P, _P], _I32),
    "wh_submit": ([_P, ctypes.POINTER(wh_request), ctypes.POINTER(_U64)], _I32),
    "wh_poll": ([_P, _U64, ctypes.POINTER(wh_result)], _I32),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_sig)


def _check(st: int, where: str) -> int:
    if st < 0:
        raise WhError(st, where)
    return st


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dptr(t: torch.Tensor, dtype=None, name: str = "tensor") -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def wh_status_str(st: int) -> str:
    return _lib.wh_status_str(st).decode()


def wh_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_lib.wh_create(device, hbm_budget_bytes, ctypes.byref(h)), "wh_create")
    return h.value


# Device buffers lent to the library (WH_DEVICE) stay referenced here until
# their matrix is unloaded or the context destroyed, so that torch's caching
# allocator cannot hand the memory to another tensor while the library still
# reads it.
_borrowed: dict = {}
# (ctx, mat) -> (rows, cols): lets the wrappers check buffer sizes, which the
# C ABI cannot see behind its raw pointers
_shapes: dict = {}


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _need(ok: bool, what: str) -> None:
    if not ok:
        raise ValueError(what)


def wh_destroy(ctx: int) -> None:
    _check(_lib.wh_destroy(ctx), "wh_destroy")
    for key in [k for k in _borrowed if k[0] == ctx]:
        del _borrowed[key]
    for key in [k for k in _shapes if k[0] == ctx]:
        del _shapes[key]


def wh_storage_bytes(rows: int, cols: int, fmt: int, rate: int = 0) -> int:
    d = wh_matrix_desc(rows, cols, fmt, rate)
    n = _U64()
    _check(_lib.wh_storage_bytes(ctypes.byref(d), ctypes.byref(n)), "wh_storage_bytes")
    return n.value


def wh_load_compressed(ctx: int, rows: int, cols: int, fmt: int, rate: int, data) -> int:
    """`data`: a CUDA tensor (borrowed: the binding keeps a reference until
    wh_unload / wh_destroy; do not modify it meanwhile) or a host numpy/CPU
    tensor (copied).  Returns the matrix handle."""
    d = wh_matrix_desc(rows, cols, fmt, rate)
    h = _U64()
    if isinstance(data, torch.Tensor) and data.is_cuda:
        ptr, nbytes, where = _dptr(data, name="data"), data.numel() * data.element_size(), WH_DEVICE
    else:
        import numpy as np
        arr = data.numpy() if isinstance(data, torch.Tensor) else data
        arr = np.ascontiguousarray(arr)
        ptr, nbytes, where = arr.ctypes.data, arr.nbytes, WH_HOST
    _check(_lib.wh_load_compressed(ctx, ctypes.byref(d), ptr, nbytes, where, ctypes.byref(h)), "wh_load_compressed")
    if where == WH_DEVICE:
        _borrowed[(ctx, h.value)] = data
    _shapes[(ctx, h.value)] = (rows, cols)
    return h.value


def wh_unload(ctx: int, mat: int) -> None:
    _check(_lib.wh_unload(ctx, mat), "wh_unload")
    _shapes.pop((ctx, mat), None)
    # wh_unload frees after pending work on the library's side; a borrowed
    # buffer may still be read by work queued on the caller's streams, so
    # release it only once the device is idle
    if (ctx, mat) in _borrowed:
        torch.cuda.synchronize()
        del _borrowed[(ctx, mat)]


def wh_gemv(ctx: int, mat: int, u: torch.Tensor, y: torch.Tensor, row_begin: int, row_end: int,
            flags: int = WH_ACC_DEFAULT, stream=None) -> None:
    shp = _shapes.get((ctx, mat))
    if shp is not None:
        _need(u.numel() >= shp[1], f"u holds {u.numel()} values, the matrix has {shp[1]} columns")
        _need(y.numel() >= row_end - row_begin, f"y holds {y.numel()} values for {row_end - row_begin} rows")
    _check(_lib.wh_gemv(ctx, mat, _dptr(u, torch.float32, "u"), _dptr(y, torch.float32, "y"), row_begin, row_end,
                        flags, _stream(stream)), "wh_gemv")


def wh_gemv_noalloc(ctx: int, mat: int, u: torch.Tensor, y: torch.Tensor, row_begin: int, row_end: int,
                    flags: int = WH_ACC_DEFAULT, stream=None) -> None:
    shp = _shapes.get((ctx, mat))
    if shp is not None:
        _need(u.numel() >= shp[1], f"u holds {u.numel()} values, the matrix has {shp[1]} columns")
        _need(y.numel() >= row_end - row_begin, f"y holds {y.numel()} values for {row_end - row_begin} rows")
    _check(_lib.wh_gemv_noalloc(ctx, mat, _dptr(u, torch.float32, "u"), _dptr(y, torch.float32, "y"), row_begin,
                                row_end, flags, _stream(stream)), "wh_gemv_noalloc")


def wh_gemv_host(ctx: int, h_code, rows: int, cols: int, rate: int, u: torch.Tensor, y: torch.Tensor,
                 row_begin: int = 0, row_end: int | None = None, chunk_rows: int = 0, flags: int = WH_ACC_DEFAULT,
                 stream=None) -> None:
    """y = M[row_begin:row_end] u for a WHZ1 matrix held in host memory.
    `h_code`: the whole stream as a CPU uint8 tensor (page-locked for
    overlapped copies) or a numpy array.  The binding keeps a reference to
    the latest `h_code` of each context; the caller keeps it unchanged until
    the work on `stream` has finished."""
    import numpy as np
    row_end = rows if row_end is None else row_end
    if isinstance(h_code, torch.Tensor):
        if h_code.is_cuda or not h_code.is_contiguous():
            raise TypeError("h_code must be a contiguous CPU tensor or a numpy array")
        ptr, nbytes = h_code.data_ptr(), _nbytes(h_code)
    else:
        if not isinstance(h_code, np.ndarray) or not h_code.flags.c_contiguous:
            raise TypeError("h_code must be a contiguous CPU tensor or a numpy array")
        ptr, nbytes = h_code.ctypes.data, h_code.nbytes
    _need(nbytes >= stream_bytes(rows, cols, rate),
          f"h_code holds {nbytes} bytes, the code takes {stream_bytes(rows, cols, rate)}")
    _need(u.numel() >= cols, f"u holds {u.numel()} values, the matrix has {cols} columns")
    _need(y.numel() >= max(row_end - row_begin, 0), f"y holds {y.numel()} values for {row_end - row_begin} rows")
    _borrowed[(ctx, "host_code")] = h_code
    _check(_lib.wh_gemv_host(ctx, ptr, rows, cols, rate, _dptr(u, torch.float32, "u"), _dptr(y, torch.float32, "y"),
                             row_begin, row_end, chunk_rows, flags, _stream(stream)), "wh_gemv_host")


def wh_encode_var(M, fmt: int, rate: int):
    """Host encoder of the variable-rate formats: M (rows, cols) float32
    numpy -> the storage bytes (uint8 numpy) for wh_load_compressed."""
    import numpy as np
    M = np.ascontiguousarray(M, dtype=np.float32)
    rows, cols = M.shape
    cap = int(_lib.wh_var_capacity_bytes(rows, cols))
    out = np.empty(cap, dtype=np.uint8)
    n = _U64()
    _check(_lib.wh_encode_var(M.ctypes.data, rows, cols, fmt, rate, out.ctypes.data, cap, ctypes.byref(n)),
           "wh_encode_var")
    return out[: n.value].copy()


def wh_gemv_plan_info(rows: int, cols: int, row_begin: int = 0, row_end: int | None = None,
                      num_cus: int = 256, rate: int = 8) -> dict:
    row_end = rows if row_end is None else row_end
    out = (_U32 * 9)()
    _check(_lib.wh_gemv_plan_info(rows, cols, row_begin, row_end, num_cus, rate, out), "wh_gemv_plan_info")
    keys = ("lanes", "rows_per_group", "ntiles", "nslab", "slab_bc", "bi_begin", "bi_end", "skip", "wg_lanes")
    return dict(zip(keys, [int(x) for x in out]))


def wh_var_index_bytes(rows: int, cols: int) -> int:
    return int(_lib.wh_var_index_bytes(rows, cols))


class HostBuffer:
    """Page-locked host memory from wh_host_alloc, viewed as a uint8 numpy
    array (`.array`); freed by close() or when collected."""

    def __init__(self, nbytes: int):
        import numpy as np
        p = ctypes.c_void_p()
        _check(_lib.wh_host_alloc(nbytes, ctypes.byref(p)), "wh_host_alloc")
        self._ptr = p.value
        self.nbytes = nbytes
        self.array = np.ctypeslib.as_array((ctypes.c_uint8 * nbytes).from_address(self._ptr))

    def close(self) -> None:
        if self._ptr:
            self.array = None
            _check(_lib.wh_host_free(self._ptr), "wh_host_free")
            self._ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ThermalSystem:
    """A (CSR) and the diagonal of B of Eq. 1, resident on the device."""

    def __init__(self, row_ptr, col, val, b, device="cuda"):
        import numpy as np
        self.n = len(row_ptr) - 1
        self.nnz = int(row_ptr[-1])
        if len(col) != self.nnz or len(val) != self.nnz or len(b) != self.n:
            raise ValueError("CSR arrays do not match: need row_ptr[n+1], col[nnz], val[nnz], b[n]")
        self.row_ptr = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.uint32).view(np.int32)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(col, dtype=np.uint32).view(np.int32)).to(device)
        self.val = torch.from_numpy(np.ascontiguousarray(val, dtype=np.float32)).to(device)
        self.b = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).to(device)


def wh_thermal_step(ctx: int, sysm: ThermalSystem, T: torch.Tensor, u: torch.Tensor, T_next: torch.Tensor,
                    stream=None) -> None:
    for name, t in (("T", T), ("u", u), ("T_next", T_next)):
        _need(t.numel() >= sysm.n, f"{name} holds {t.numel()} values for {sysm.n} temperatures")
    _check(_lib.wh_thermal_step(ctx, sysm.n, sysm.nnz, sysm.row_ptr.data_ptr(), sysm.col.data_ptr(),
                                sysm.val.data_ptr(), sysm.b.data_ptr(), _dptr(T, torch.float32, "T"),
                                _dptr(u, torch.float32, "u"), _dptr(T_next, torch.float32, "T_next"),
                                _stream(stream)), "wh_thermal_step")


def wh_thermal_run(ctx: int, sysm: ThermalSystem, T: torch.Tensor, U: torch.Tensor, work: torch.Tensor,
                   stream=None) -> None:
    """U: (steps, ldu >= n) float32, rows contiguous; T updated in place."""
    if U.dim() != 2 or U.stride(1) != 1:
        raise ValueError("U must be (steps, ldu) with contiguous rows")
    _need(U.shape[1] >= sysm.n, f"rows of U hold {U.shape[1]} values for {sysm.n} temperatures")
    for name, t in (("T", T), ("work", work)):
        _need(t.numel() >= sysm.n, f"{name} holds {t.numel()} values for {sysm.n} temperatures")
    _check(_lib.wh_thermal_run(ctx, sysm.n, sysm.nnz, sysm.row_ptr.data_ptr(), sysm.col.data_ptr(),
                               sysm.val.data_ptr(), sysm.b.data_ptr(), _dptr(T, torch.float32, "T"),
                               _dptr(U, torch.float32, "U"), U.stride(0), U.shape[0],
                               _dptr(work, torch.float32, "work"), _stream(stream)), "wh_thermal_run")


def wh_gemv_batched(ctx: int, mat: int, U: torch.Tensor, Y: torch.Tensor, flags: int = WH_ACC_DEFAULT,
                    stream=None) -> None:
    """U: (k, ldu >= cols) float32 or bfloat16; Y: (k, ldy >= rows) float32;
    rows of both contiguous."""
    if U.dim() != 2 or Y.dim() != 2 or U.shape[0] != Y.shape[0]:
        raise ValueError("U and Y must be (k, n) with the same k")
    if not (U.is_cuda and Y.is_cuda) or Y.dtype != torch.float32:
        raise TypeError("U and Y must be CUDA tensors; Y float32")
    if U.dtype == torch.float32:
        dt = WH_U_F32
    elif U.dtype == torch.bfloat16:
        dt = WH_U_BF16
    else:
        raise TypeError("U must be float32 or bfloat16")
    if U.stride(1) != 1 or Y.stride(1) != 1:
        raise ValueError("rows of U and Y must be contiguous")
    _check(_lib.wh_gemv_batched(ctx, mat, U.data_ptr(), dt, U.shape[0], U.stride(0), Y.data_ptr(), Y.stride(0),
                                flags, _stream(stream)), "wh_gemv_batched")


def wh_decode_debug(ctx: int, mat: int, block_begin: int, nblocks: int, out: torch.Tensor, stream=None) -> None:
    _need(out.numel() >= 16 * nblocks, f"out holds {out.numel()} values for {nblocks} blocks")
    _check(_lib.wh_decode_debug(ctx, mat, block_begin, nblocks, _dptr(out, torch.float32, "out"), _stream(stream)),
           "wh_decode_debug")


def wh_decode(ctx: int, mat: int, out: torch.Tensor, stream=None) -> None:
    shp = _shapes.get((ctx, mat))
    if shp is not None:
        _need(out.numel() >= shp[0] * shp[1], f"out holds {out.numel()} values for a {shp[0]} x {shp[1]} matrix")
    _check(_lib.wh_decode(ctx, mat, _dptr(out, torch.float32, "out"), _stream(stream)), "wh_decode")


def wh_encode(ctx: int, M: torch.Tensor, rate: int, stream_out: torch.Tensor, bad: torch.Tensor | None = None,
              stream=None) -> None:
    rows, cols = M.shape
    _need(_nbytes(stream_out) >= stream_bytes(rows, cols, rate),
          f"stream_out holds {_nbytes(stream_out)} bytes, the code takes {stream_bytes(rows, cols, rate)}")
    _check(_lib.wh_encode(ctx, _dptr(M, torch.float32, "M"), rows, cols, rate, _dptr(stream_out, name="stream_out"),
                          None if bad is None else _dptr(bad, torch.int32, "bad"), _stream(stream)), "wh_encode")


def wh_quantize(ctx: int, M: torch.Tensor, fmt: int, out: torch.Tensor, stream=None) -> None:
    rows, cols = M.shape
    _need(_nbytes(out) >= wh_storage_bytes(rows, cols, fmt),
          f"out holds {_nbytes(out)} bytes, the format takes {wh_storage_bytes(rows, cols, fmt)}")
    _check(_lib.wh_quantize(ctx, _dptr(M, torch.float32, "M"), rows, cols, fmt, _dptr(out, name="out"),
                            _stream(stream)), "wh_quantize")


def wh_stream_read(ctx: int, buf: torch.Tensor, out: torch.Tensor, stream=None) -> None:
    nbytes = buf.numel() * buf.element_size()
    _check(_lib.wh_stream_read(ctx, _dptr(buf, name="buf"), nbytes, _dptr(out, torch.int32, "out"), _stream(stream)),
           "wh_stream_read")


def wh_submit(ctx: int, req: wh_request) -> int:
    t = _U64()
    _check(_lib.wh_submit(ctx, ctypes.byref(req), ctypes.byref(t)), "wh_submit")
    return t.value


def wh_poll(ctx: int, ticket: int) -> tuple[int, wh_result]:
    r = wh_result()
    st = _check(_lib.wh_poll(ctx, ticket, ctypes.byref(r)), "wh_poll")
    return st, r


# ------------------------------------------------------------- convenience
@dataclass
class Matrix:
    ctx: int
    handle: int
    rows: int
    cols: int
    fmt: int
    rate: int
    storage: object  # keeps a borrowed device buffer alive


def stream_bytes(rows: int, cols: int, rate: int) -> int:
    return wh_storage_bytes(rows, cols, WH_FMT_ZFP_FIXED_RATE, rate)
