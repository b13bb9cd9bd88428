"""GPU parity of the dense reduced-precision storage path (precision sweep).

  codes     the library's quantisers (FP16 / BF16 RNE, FP8 e4m3 + per-block
            FP32 scale) produce the oracle's codes bit for bit
  decode    the hardware e4m3 -> FP32 conversion gives the format's value
            for every non-NaN code
  gemv      relative L2 of y against the FP64 product with the FP32 source
            matrix: 1e-6 (FP32), 2e-3 (FP16, BF16), 2e-2 (FP8 + scale); and
            within 1e-6 of the FP64 product with the dequantised matrix, so
            the kernel arithmetic is checked apart from the quantisation
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import quant
from paper_1902_08018_amd import synth, wh

pytestmark = pytest.mark.gpu

TOL = {wh.WH_FMT_F32: 1e-6, wh.WH_FMT_F16: 2e-3, wh.WH_FMT_BF16: 2e-3, wh.WH_FMT_FP8E4M3_BS4: 2e-2}
NAMES = {wh.WH_FMT_F32: "f32", wh.WH_FMT_F16: "f16", wh.WH_FMT_BF16: "bf16", wh.WH_FMT_FP8E4M3_BS4: "fp8bs"}


def rel_l2(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def quantize_gpu(ctx, M, fmt):
    rows, cols = M.shape
    Md = torch.from_numpy(np.ascontiguousarray(M, dtype=np.float32)).cuda()
    if fmt == wh.WH_FMT_F32:
        return Md.view(-1)
    out = torch.zeros(wh.wh_storage_bytes(rows, cols, fmt), dtype=torch.uint8, device="cuda")
    wh.wh_quantize(ctx, Md, fmt, out)
    torch.cuda.synchronize()
    return out


def dequantized(M, fmt):
    rows, cols = M.shape
    if fmt == wh.WH_FMT_F32:
        return M.astype(np.float64)
    if fmt == wh.WH_FMT_F16:
        return quant.to_f16(M).astype(np.float64)
    if fmt == wh.WH_FMT_BF16:
        return quant.bf16_values(quant.bf16_bits(M)).astype(np.float64)
    codes, scales = quant.fp8_block_scaled(M)
    return quant.fp8_dequant(codes, scales, rows, cols)


@pytest.fixture(scope="module")
def small_dense():
    M = synth.matrix(synth.SMALL)
    u = synth.u_vector(synth.SMALL)
    return M, u, oracle.dense_gemv_fp64(M, u)


def test_quantizer_codes_bitexact(gpu_ctx):
    spec = synth.MatrixSpec(256, 1024, 32, 8.0, seed=11)
    M = synth.matrix(spec)
    M[:4, :4] = 0.0  # a zero block
    M[8:12, 8:12] *= -1e-30  # tiny block
    f16 = quantize_gpu(gpu_ctx, M, wh.WH_FMT_F16).cpu().numpy().view(np.uint16)
    assert np.array_equal(f16, quant.to_f16(M).view(np.uint16).reshape(-1))
    bf = quantize_gpu(gpu_ctx, M, wh.WH_FMT_BF16).cpu().numpy().view(np.uint16)
    assert np.array_equal(bf, quant.bf16_bits(M).reshape(-1))
    raw = quantize_gpu(gpu_ctx, M, wh.WH_FMT_FP8E4M3_BS4).cpu().numpy()
    nb = M.size // 16
    codes, scales = quant.fp8_block_scaled(M)
    assert np.array_equal(raw[:nb * 16].reshape(nb, 16), codes)
    assert np.array_equal(raw[nb * 16:].view(np.float32), scales)


def test_fp8_hardware_decode_every_code(gpu_ctx):
    """y = M e_j reads column j of a one-block-row FP8 matrix with unit
    scales: each of the 254 non-NaN codes must decode to its e4m3 value."""
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)] + [0, 0], dtype=np.uint8)  # 256 codes
    nblk = 16
    blocks = codes.reshape(nblk, 16)
    raw = np.concatenate([blocks.reshape(-1), np.ones(nblk, dtype=np.float32).view(np.uint8)])
    mat = wh.wh_load_compressed(gpu_ctx, 4, 4 * nblk, wh.WH_FMT_FP8E4M3_BS4, 0, raw)
    y = torch.empty(4, dtype=torch.float32, device="cuda")
    got = np.zeros((nblk, 16))
    for j in range(4 * nblk):
        u = torch.zeros(4 * nblk, dtype=torch.float32, device="cuda")
        u[j] = 1.0
        wh.wh_gemv(gpu_ctx, mat, u, y, 0, 4)
        yy = y.cpu().numpy()
        b, c = divmod(j, 4)
        for r in range(4):
            got[b, 4 * r + c] = yy[r]
    want = quant.E4M3_TABLE[blocks.astype(np.int64)]
    assert np.array_equal(got, want)
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("fmt", [wh.WH_FMT_F32, wh.WH_FMT_F16, wh.WH_FMT_BF16, wh.WH_FMT_FP8E4M3_BS4])
@pytest.mark.parametrize("flags", [wh.WH_ACC_DEFAULT, wh.WH_ACC_TWOSUM])
def test_dense_gemv_small_config(gpu_ctx, small_dense, fmt, flags):
    M, u, ref_src = small_dense
    store = quantize_gpu(gpu_ctx, M, fmt)
    mat = wh.wh_load_compressed(gpu_ctx, 4096, 4096, fmt, 0, store)
    y = torch.empty(4096, dtype=torch.float32, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u).cuda(), y, 0, 4096, flags)
    torch.cuda.synchronize()
    g = y.cpu().numpy()
    err_src = rel_l2(g, ref_src)
    ref_q = dequantized(M, fmt) @ u.astype(np.float64)
    err_q = rel_l2(g, ref_q)
    print(f"{NAMES[fmt]} flags {flags}: rel-L2 vs FP32-source FP64 {err_src:.3e}, vs dequantised {err_q:.3e}")
    assert err_src <= TOL[fmt]
    assert err_q <= 1e-6
    # a row range (slit rows of the field matrix)
    y2 = torch.empty(1020, dtype=torch.float32, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u).cuda(), y2, 2048, 3068, flags)
    torch.cuda.synchronize()
    assert rel_l2(y2.cpu().numpy(), ref_q[2048:3068]) <= 1e-6
    # a range that starts and ends inside block rows: row-major storage takes
    # it; block-scaled FP8 works on whole 4 x 4 tiles and rejects it
    if fmt == wh.WH_FMT_FP8E4M3_BS4:
        with pytest.raises(wh.WhError) as ei:
            wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u).cuda(), y2, 2049, 3067, flags)
        assert ei.value.status == wh.WH_ERR_SHAPE
    else:
        y3 = torch.full((1020,), -7.0, dtype=torch.float32, device="cuda")
        wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u).cuda(), y3, 2049, 3067, flags)
        torch.cuda.synchronize()
        y3h = y3.cpu().numpy()
        assert rel_l2(y3h[:1018], ref_q[2049:3067]) <= 1e-6
        assert np.all(y3h[1018:] == -7.0)
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("shape", [(4, 8), (260, 1032), (1028, 264), (12, 65544)])
@pytest.mark.parametrize("fmt", [wh.WH_FMT_F32, wh.WH_FMT_BF16, wh.WH_FMT_FP8E4M3_BS4])
def test_dense_gemv_ragged(gpu_ctx, shape, fmt):
    rows, cols = shape
    spec = synth.MatrixSpec(rows, cols, 64, 8.0, seed=5)
    M = synth.matrix(spec)
    u = synth.uniform(cols, seed=5)
    store = quantize_gpu(gpu_ctx, M, fmt)
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, fmt, 0, store)
    y = torch.empty(rows, dtype=torch.float32, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u).cuda(), y, 0, rows)
    torch.cuda.synchronize()
    err = rel_l2(y.cpu().numpy(), dequantized(M, fmt) @ u.astype(np.float64))
    assert err <= 1e-6
    wh.wh_unload(gpu_ctx, mat)


def test_dense_f32_paper_mp(gpu_ctx, small_dense):
    M, u, _ = small_dense
    ref = oracle.dense_gemv_paper_mp(M, u)
    store = quantize_gpu(gpu_ctx, M, wh.WH_FMT_F32)
    mat = wh.wh_load_compressed(gpu_ctx, 4096, 4096, wh.WH_FMT_F32, 0, store)
    y = torch.empty(4096, dtype=torch.float32, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, torch.from_numpy(u).cuda(), y, 0, 4096, wh.WH_PAPER_MP)
    torch.cuda.synchronize()
    g = y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - ref) <= np.spacing(np.abs(ref).astype(np.float32)))
    with pytest.raises(wh.WhError):
        bf = quantize_gpu(gpu_ctx, M, wh.WH_FMT_BF16)
        m2 = wh.wh_load_compressed(gpu_ctx, 4096, 4096, wh.WH_FMT_BF16, 0, bf)
        wh.wh_gemv(gpu_ctx, m2, torch.from_numpy(u).cuda(), y, 0, 4096, wh.WH_PAPER_MP)
    wh.wh_unload(gpu_ctx, mat)
