"""GPU parity of the variable-rate formats (fixed precision, fixed accuracy;
Sec. 4.3, Table 2) against the oracle.

  decode   wh_decode bit-exact against the oracle's decode (both from the
           same bytes: the library's host encoder, itself bit-equal to the
           oracle's on the CPU), partial edge blocks, groups of 32 blocks cut
           by the matrix edge
  GEMV     the fused decode + GEMV within 1e-6 relative L2 of the FP64 GEMV
           of the oracle-decoded matrix, on row ranges that start and end
           inside block rows, FP64 and TwoSum accumulation, 1 to 8 lanes per
           block row (the number of 32-block groups in a row)
  large    2^18 lanes and more (the 1024-lane workgroups): decode bit-exact
           and the GEMV on sampled bands of block rows
  errors   Fig. 7 mode, batched products and short storage are refused
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1902_08018_amd import synth, wh

pytestmark = pytest.mark.gpu

CASES = [(wh.WH_FMT_ZFP_FIXED_PRECISION, 17), (wh.WH_FMT_ZFP_FIXED_PRECISION, 6),
         (wh.WH_FMT_ZFP_FIXED_ACCURACY, -20), (wh.WH_FMT_ZFP_FIXED_ACCURACY, -10)]
SHAPES = [(1, 1), (7, 13), (130, 378), (378, 1030), (61, 4100), (1030, 6)]


def rel_l2(y, ref):
    y = np.asarray(y, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))


def setup(rows, cols, fmt, param, seed=21):
    spec = synth.MatrixSpec(rows, cols, 32, 8.0, seed=seed)
    M = synth.matrix(spec)
    rate = param if fmt == wh.WH_FMT_ZFP_FIXED_PRECISION else wh.accuracy_rate(param)
    omode = oracle.VAR_PRECISION if fmt == wh.WH_FMT_ZFP_FIXED_PRECISION else oracle.VAR_ACCURACY
    buf = wh.wh_encode_var(M, fmt, rate)
    ib = wh.wh_var_index_bytes(rows, cols)
    want = oracle.decode_var(buf[ib:], buf[:ib].view(np.uint64), rows, cols, omode, param)
    return M, rate, buf, want


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("fmt,param", CASES)
def test_decode_bitexact(gpu_ctx, shape, fmt, param):
    rows, cols = shape
    M, rate, buf, want = setup(rows, cols, fmt, param)
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, fmt, rate, buf)
    out = torch.full((rows + 1, cols), -7.0, device="cuda")
    wh.wh_decode(gpu_ctx, mat, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got[:rows].view(np.uint32), want.view(np.uint32))
    assert np.all(got[rows:] == -7.0)
    if fmt == wh.WH_FMT_ZFP_FIXED_ACCURACY:
        assert float(np.abs(want.astype(np.float64) - M).max()) <= 2.0 ** param
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("fmt,param", CASES)
def test_gemv(gpu_ctx, shape, fmt, param):
    rows, cols = shape
    M, rate, buf, want = setup(rows, cols, fmt, param, seed=22)
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, fmt, rate, buf)
    u_np = synth.uniform(cols, seed=23)
    u = torch.from_numpy(u_np).cuda()
    ref = want.astype(np.float64) @ u_np.astype(np.float64)
    for flags in (wh.WH_ACC_DEFAULT, wh.WH_ACC_TWOSUM):
        for rb, re in [(0, rows), (rows // 3, rows - rows // 4), (rows - 1, rows), (1, 2)]:
            if not 0 <= rb < re <= rows:
                continue
            y = torch.full((re - rb + 2,), -7.0, device="cuda")
            wh.wh_gemv(gpu_ctx, mat, u, y, rb, re, flags)
            torch.cuda.synchronize()
            yh = y.cpu().numpy()
            assert rel_l2(yh[:re - rb], ref[rb:re]) <= 1e-6, (flags, rb, re)
            assert np.all(yh[re - rb:] == -7.0)
    wh.wh_unload(gpu_ctx, mat)


# 2^18 lanes (one per block row and 32-block group) and more take the
# 1024-lane workgroups; the oracle decodes sampled bands of block rows from
# the index, among them the first, the last and bands across workgroup tiles
# (16 block rows per decode workgroup, 128 per GEMV tile at 8 lanes a row)
@pytest.mark.parametrize("rows,cols,fmt,param", [(16382, 8190, wh.WH_FMT_ZFP_FIXED_PRECISION, 17),
                                                 (16384, 8192, wh.WH_FMT_ZFP_FIXED_ACCURACY, -20)])
def test_large_launch_sampled(gpu_ctx, rows, cols, fmt, param):
    M = synth.matrix(synth.MatrixSpec(rows, cols, 32, 8.0, seed=24))
    rate = param if fmt == wh.WH_FMT_ZFP_FIXED_PRECISION else wh.accuracy_rate(param)
    omode = oracle.VAR_PRECISION if fmt == wh.WH_FMT_ZFP_FIXED_PRECISION else oracle.VAR_ACCURACY
    buf = wh.wh_encode_var(M, fmt, rate)
    ib = wh.wh_var_index_bytes(rows, cols)
    index = buf[:ib].view(np.uint64)
    nbr, ng = (rows + 3) // 4, ((cols + 3) // 4 + 31) // 32
    assert nbr * ng >= 1 << 18
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, fmt, rate, buf)
    out = torch.empty((rows, cols), device="cuda")
    wh.wh_decode(gpu_ctx, mat, out)
    u_np = synth.uniform(cols, seed=25)
    y = torch.full((rows + 2,), -7.0, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u_np).cuda(), y, 0, rows, wh.WH_ACC_DEFAULT)
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    assert np.all(yh[rows:] == -7.0)
    for b0, b1 in [(0, 20), (120, 136), (1010, 1030), (2047, 2049), (nbr - 20, nbr)]:
        r0, r1 = 4 * b0, min(4 * b1, rows)
        want = oracle.decode_var(buf[ib:], index[b0 * ng:b1 * ng], r1 - r0, cols, omode, param)
        got = out[r0:r1].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (b0, b1)
        ref = want.astype(np.float64) @ u_np.astype(np.float64)
        assert rel_l2(yh[r0:r1], ref) <= 1e-6, (b0, b1)
    wh.wh_unload(gpu_ctx, mat)


def test_refusals(gpu_ctx):
    rows, cols = 64, 256
    M, rate, buf, want = setup(rows, cols, wh.WH_FMT_ZFP_FIXED_PRECISION, 12)
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_PRECISION, 12, buf)
    u = torch.rand(cols, device="cuda")
    y = torch.empty(rows, device="cuda")
    with pytest.raises(wh.WhError) as ei:
        wh.wh_gemv(gpu_ctx, mat, u, y, 0, rows, wh.WH_PAPER_MP)
    assert ei.value.status == wh.WH_ERR_FORMAT
    with pytest.raises(wh.WhError) as ei:
        wh.wh_gemv_batched(gpu_ctx, mat, torch.rand((4, cols), device="cuda"), torch.empty((4, rows), device="cuda"))
    assert ei.value.status == wh.WH_ERR_FORMAT
    wh.wh_unload(gpu_ctx, mat)
    ib = wh.wh_var_index_bytes(rows, cols)
    with pytest.raises(wh.WhError) as ei:
        wh.wh_load_compressed(gpu_ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_PRECISION, 12, buf[:ib + 8])
    assert ei.value.status == wh.WH_ERR_FORMAT
    with pytest.raises(wh.WhError) as ei:
        wh.wh_load_compressed(gpu_ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_PRECISION, 40, buf)
    assert ei.value.status == wh.WH_ERR_FORMAT
