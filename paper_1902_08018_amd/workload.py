"""Resident compressed matrices for the benchmarks and GPU tests.

Builds a WHZ1 stream of a synthetic response matrix directly in device
memory: rows of the FP32 matrix are generated on the GPU a chunk at a time
(`synth`), and the library's GPU encoder (`wh_encode`) writes the matching
slice of the stream.  The dense FP32 matrix is never held whole.
"""
from __future__ import annotations

import torch

from . import synth
from . import wh


def build_stream(ctx: int, spec: synth.MatrixSpec, rate: int, chunk_rows: int = 4096,
                 device: str = "cuda") -> torch.Tensor:
    """Device uint8 tensor holding the rate-`rate` stream of `spec`."""
    nbytes = wh.stream_bytes(spec.rows, spec.cols, rate)
    out = torch.empty(nbytes, dtype=torch.uint8, device=device)
    table = synth.device_table(spec, device)
    chunk_rows = max(4, min(chunk_rows, spec.rows) // 4 * 4)
    scratch = torch.empty(chunk_rows * spec.cols, dtype=torch.float32, device=device)
    bad = torch.zeros(1, dtype=torch.int32, device=device)
    per_block_row = wh.stream_bytes(4, spec.cols, rate)  # bytes of stream per 4 matrix rows
    for r0 in range(0, spec.rows, chunk_rows):  # chunks start on block-rows; the last may be partial
        r1 = min(spec.rows, r0 + chunk_rows)
        m = scratch[: (r1 - r0) * spec.cols]
        synth.matrix_rows_device(spec, r0, r1, m, table)
        wh.wh_encode(ctx, m.view(r1 - r0, spec.cols), rate,
                     out[r0 // 4 * per_block_row: (r1 + 3) // 4 * per_block_row], bad)
    torch.cuda.synchronize()
    if int(bad.item()) != 0:
        raise RuntimeError(f"{int(bad.item())} blocks held NaN/Inf")
    del scratch
    return out


def build_dense(spec: synth.MatrixSpec, chunk_rows: int = 4096, device: str = "cuda") -> torch.Tensor:
    """The FP32 matrix itself, (rows, cols), generated on the GPU."""
    out = torch.empty((spec.rows, spec.cols), dtype=torch.float32, device=device)
    table = synth.device_table(spec, device)
    for r0 in range(0, spec.rows, chunk_rows):
        r1 = min(spec.rows, r0 + chunk_rows)
        synth.matrix_rows_device(spec, r0, r1, out[r0:r1].view(-1), table)
    torch.cuda.synchronize()
    return out


def u_device(spec: synth.MatrixSpec, stream_id: int = synth.STREAM_U, offset: int = 0,
             device: str = "cuda") -> torch.Tensor:
    u = torch.empty(spec.cols, dtype=torch.float32, device=device)
    synth.uniform_device(u, spec.seed, stream_id, offset)
    return u
