"""Seeded synthetic inputs for the compressed-matrix GEMV.

The paper's deformation matrices C_d and temperature vectors S_k (Sec. 2.1,
Eq. 2) are not public.  The stand-in is a response matrix over two
unit-spaced g x g lattices (point i at (i mod g, i div g)):

    M[i, j] = RNE_f32( exp(-|p_i - q_j| / ell) + sigma * z_ij ),

with z_ij an Irwin-Hall(12) normal deviate from a counter-based hash
(stream 0), and dose vectors u_j = (hash >> 40) * 2^-24 uniform on [0, 1)
(stream 1; stream 2 for multi-right-hand-side batches; stream 3 for serving
traces).  Host (C) and device (HIP) implementations produce identical bits.

This module holds none of the codec or GEMV arithmetic; both the oracle side
and the GPU side take their inputs from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "csrc")
_HOST_SRC = os.path.join(_CSRC, "synth_host.c")
_HOST_LIB = os.path.join(_HERE, "libwhsynth.so")
_DEV_SRC = os.path.join(_CSRC, "synth_dev.hip")
_DEV_LIB = os.path.join(_HERE, "libwhsynth_dev.so")

STREAM_NOISE, STREAM_U, STREAM_UBATCH, STREAM_TRACE, STREAM_THERMAL = 0, 1, 2, 3, 4


@dataclass(frozen=True)
class MatrixSpec:
    """A synthetic response matrix: rows x cols over g-wide lattices."""
    rows: int
    cols: int
    g: int
    ell: float
    sigma: float = 1e-4
    seed: int = 0

    @property
    def ndy(self) -> int:
        return (max(self.rows, self.cols) + self.g - 1) // self.g


# The two plain-path workloads: 4096^2 on 64x64 lattices (ell 8) and
# 65536^2 on 256x256 lattices (ell 32); noise sigma 1e-4, seed 0.
SMALL = MatrixSpec(4096, 4096, 64, 8.0)
LARGE = MatrixSpec(65536, 65536, 256, 32.0)


def build_host(force: bool = True) -> str:
    if force or not os.path.exists(_HOST_LIB):
        tmp = _HOST_LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-o", tmp, _HOST_SRC, "-lm"])
        os.replace(tmp, _HOST_LIB)
    return _HOST_LIB


def build_device(hipcc: str = "hipcc", force: bool = True) -> str:
    if force or not os.path.exists(_DEV_LIB):
        tmp = _DEV_LIB + f".tmp{os.getpid()}"
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-ffp-contract=off",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-o", tmp, _DEV_SRC], stderr=subprocess.DEVNULL)
        os.replace(tmp, _DEV_LIB)
    return _DEV_LIB


_host = None
_dev = None


def _hostlib():
    global _host
    if _host is None:
        if not os.path.exists(_HOST_LIB):
            build_host()
        L = ctypes.CDLL(_HOST_LIB)
        P, U32, U64, D = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.whs_hash.argtypes = [U64, U32, U64]
        L.whs_hash.restype = U64
        L.whs_kernel_table.argtypes = [U32, U32, D, P]
        L.whs_matrix_rows.argtypes = [U64, U32, U32, D, P, U32, U32, P]
        L.whs_uniform.argtypes = [U64, U32, U64, U64, P]
        _host = L
    return _host


def _devlib():
    global _dev
    if _dev is None:
        if not os.path.exists(_DEV_LIB):
            raise RuntimeError(f"device generator not built: {_DEV_LIB} (run __graft_entry__.build())")
        import torch  # noqa: F401  (load torch's HIP runtime first)
        L = ctypes.CDLL(_DEV_LIB)
        P, U32, U64, D = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.whs_dev_matrix_rows.argtypes = [U64, U32, U32, D, P, U32, U32, P, P]
        L.whs_dev_matrix_rows.restype = ctypes.c_int
        L.whs_dev_uniform.argtypes = [U64, U32, U64, U64, P, P]
        L.whs_dev_uniform.restype = ctypes.c_int
        _dev = L
    return _dev


def hash64(seed: int, stream: int, k: int) -> int:
    return int(_hostlib().whs_hash(seed, stream, k))


def kernel_table(spec: MatrixSpec) -> np.ndarray:
    t = np.empty(spec.ndy * spec.g, dtype=np.float64)
    _hostlib().whs_kernel_table(spec.g, spec.ndy, spec.ell, t.ctypes.data)
    return t


def matrix_rows(spec: MatrixSpec, r0: int, r1: int, table: np.ndarray | None = None) -> np.ndarray:
    """Rows [r0, r1) of the matrix as float32 (r1 - r0, cols), on the host."""
    assert 0 <= r0 <= r1 <= spec.rows
    table = kernel_table(spec) if table is None else table
    out = np.empty((r1 - r0, spec.cols), dtype=np.float32)
    _hostlib().whs_matrix_rows(spec.seed, spec.g, spec.cols, spec.sigma, table.ctypes.data, r0, r1,
                               out.ctypes.data)
    return out


def matrix(spec: MatrixSpec) -> np.ndarray:
    return matrix_rows(spec, 0, spec.rows)


def uniform(n: int, seed: int = 0, stream: int = STREAM_U, offset: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _hostlib().whs_uniform(seed, stream, offset, n, out.ctypes.data)
    return out


def u_vector(spec: MatrixSpec) -> np.ndarray:
    """The dose vector u (length cols) that goes with a matrix spec."""
    return uniform(spec.cols, spec.seed, STREAM_U)


def u_batch(spec: MatrixSpec, k: int) -> np.ndarray:
    """k dose vectors (k, cols): row r is elements [r*cols, (r+1)*cols) of stream 2."""
    return uniform(k * spec.cols, spec.seed, STREAM_UBATCH).reshape(k, spec.cols)


# ------------------------------------------------------ thermal system
# Stand-in for the thermal model's matrices (Sec. 2.1, Eq. 1: A sparse, B
# diagonal, about 3.7e5 temperatures updated every millisecond), which are not
# given: an explicit one-millisecond step of heat conduction on an nx x ny
# mesh with a lumped (diagonal) heat capacity c_i in [1, 2) per cell and a
# conductance per mesh edge, insulated at the border:
#
#     A = I - dt C^-1 K,   B = dt C^-1,
#
# K the weighted graph Laplacian of the mesh.  Off-diagonal entries are
# r_ij = 0.2 * kappa_e / c_i with kappa_e in [0.5, 1) (so every diagonal entry
# stays >= 0.2), rounded once to FP32.  C A = C - dt K is symmetric, so A is
# not (unless all capacities are equal) and c^T A = c^T: heat is conserved.
# Rows list their columns in ascending order (north, west, self, east,
# south).  The source term u_k is a Gaussian dose spot that moves along the
# mesh's middle row, 3.7 cells per step.

@dataclass(frozen=True)
class ThermalSpec:
    nx: int
    ny: int
    seed: int = 0
    dt: float = 1e-3

    @property
    def n(self) -> int:
        return self.nx * self.ny


# about 3.7e5 temperatures, as in the paper's thermal model
THERMAL = ThermalSpec(608, 608)


def thermal_capacity(spec: ThermalSpec) -> np.ndarray:
    """c_i in [1, 2), FP64 (the generator's own value, before rounding)."""
    nh, nv = spec.ny * (spec.nx - 1), (spec.ny - 1) * spec.nx
    return 1.0 + uniform(spec.n, spec.seed, STREAM_THERMAL, nh + nv).astype(np.float64)


def thermal_system(spec: ThermalSpec):
    """CSR (row_ptr uint32 [n+1], col uint32 [nnz], val float32 [nnz]) of A
    and the diagonal of B (float32 [n])."""
    nx, ny, n = spec.nx, spec.ny, spec.n
    nh, nv = ny * (nx - 1), (ny - 1) * nx
    kh = 0.5 + 0.5 * uniform(nh, spec.seed, STREAM_THERMAL, 0).astype(np.float64)   # (x,y)-(x+1,y): y*(nx-1)+x
    kv = 0.5 + 0.5 * uniform(nv, spec.seed, STREAM_THERMAL, nh).astype(np.float64)  # (x,y)-(x,y+1): y*nx+x
    cap = thermal_capacity(spec)
    i = np.arange(n, dtype=np.int64)
    x, y = i % nx, i // nx
    has = np.stack([y > 0, x > 0, np.ones(n, bool), x < nx - 1, y < ny - 1], axis=1)
    nbr = np.stack([i - nx, i - 1, i, i + 1, i + nx], axis=1)
    kap = np.zeros((n, 5))
    kap[:, 0] = np.where(has[:, 0], kv[np.clip((y - 1) * nx + x, 0, max(nv - 1, 0))] if nv else 0.0, 0.0)
    kap[:, 1] = np.where(has[:, 1], kh[np.clip(y * (nx - 1) + x - 1, 0, max(nh - 1, 0))] if nh else 0.0, 0.0)
    kap[:, 3] = np.where(has[:, 3], kh[np.clip(y * (nx - 1) + x, 0, max(nh - 1, 0))] if nh else 0.0, 0.0)
    kap[:, 4] = np.where(has[:, 4], kv[np.clip(y * nx + x, 0, max(nv - 1, 0))] if nv else 0.0, 0.0)
    r = 0.2 * kap / cap[:, None]
    r[:, 2] = 1.0 - r.sum(axis=1)
    counts = has.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    row_ptr[1:] = np.cumsum(counts)
    col = nbr[has].astype(np.uint32)
    val = r[has].astype(np.float32)
    b = (spec.dt / cap).astype(np.float32)
    return row_ptr, col, val, b


def thermal_source(spec: ThermalSpec, step: int, sigma: float = 12.0) -> np.ndarray:
    """u_k (float32 [n]): a unit Gaussian spot centred at
    (3.7 k mod nx, ny / 2)."""
    i = np.arange(spec.n, dtype=np.int64)
    x, y = (i % spec.nx).astype(np.float64), (i // spec.nx).astype(np.float64)
    cx, cy = (3.7 * step) % spec.nx, spec.ny / 2.0
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * sigma * sigma)).astype(np.float32)


def thermal_initial(spec: ThermalSpec) -> np.ndarray:
    """T_0 (float32 [n]): 20 plus a small seeded ripple."""
    return (20.0 + 0.01 * uniform(spec.n, spec.seed, STREAM_THERMAL, 1 << 40).astype(np.float64)).astype(np.float32)


# ---------------------------------------------------------------- device
def device_table(spec: MatrixSpec, device="cuda"):
    import torch
    return torch.from_numpy(kernel_table(spec)).to(device)


def matrix_rows_device(spec: MatrixSpec, r0: int, r1: int, out, d_table, stream=None) -> None:
    """Fill the float32 CUDA tensor `out` ((r1-r0)*cols elements) on the GPU."""
    import torch
    assert out.dtype == torch.float32 and out.is_cuda and out.is_contiguous()
    assert out.numel() == (r1 - r0) * spec.cols
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    st = _devlib().whs_dev_matrix_rows(spec.seed, spec.g, spec.cols, spec.sigma, d_table.data_ptr(), r0, r1,
                                       out.data_ptr(), s)
    if st != 0:
        raise RuntimeError(f"whs_dev_matrix_rows failed ({st})")


def uniform_device(out, seed: int = 0, stream_id: int = STREAM_U, offset: int = 0, stream=None) -> None:
    import torch
    assert out.dtype == torch.float32 and out.is_cuda and out.is_contiguous()
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    st = _devlib().whs_dev_uniform(seed, stream_id, offset, out.numel(), out.data_ptr(), s)
    if st != 0:
        raise RuntimeError(f"whs_dev_uniform failed ({st})")
