"""Parity of the precision sweep and of the multi-right-hand-side path at the
full 65536 x 65536 size, in the launch configuration the benchmark times
(whole matrix resident, one call over all rows).

The oracle checks sampled block rows: the host generator makes those rows of
the FP32 source matrix, and
  * dense storage (FP16 / BF16 / FP8 e4m3 + one FP32 scale per 4x4 block):
    the GPU quantiser's codes on those rows equal the oracle quantiser's bit
    for bit; y on those rows is within relative L2 2e-3 / 2e-3 / 2e-2 of the
    FP64 product with the FP32 source rows, and within 1e-6 of the FP64
    product with the oracle-dequantised rows (the kernel's arithmetic alone);
  * multi-RHS (k = 4, 16, 64; FP32 and BF16 U): Y on those rows is within
    relative L2 1e-6 (FP32 U) / 2e-3 (BF16 U) per right-hand side of the FP64
    product of the oracle-decoded rows (the oracle encodes them itself) with
    U (for BF16, with U rounded to BF16).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import quant
from paper_1902_08018_amd import synth, wh, workload

pytestmark = pytest.mark.gpu

SPEC = synth.LARGE
NBR = SPEC.rows // 4
# 32 sampled block rows: both ends, tile edges, and a spread in between
SAMPLE_BR = sorted(set([0, 1, 31, 32, 8191, 8192, NBR // 2, NBR - 2, NBR - 1]
                       + [int(x) for x in np.linspace(2, NBR - 3, 23)]))


def rel_l2(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module")
def source_rows():
    table = synth.kernel_table(SPEC)
    return {bi: synth.matrix_rows(SPEC, 4 * bi, 4 * bi + 4, table) for bi in SAMPLE_BR}


def test_dense_precision_sweep_full_size(gpu_ctx, source_rows):
    rows, cols = SPEC.rows, SPEC.cols
    dense = workload.build_dense(SPEC)
    u_host = synth.u_vector(SPEC)
    u = workload.u_device(SPEC)
    assert np.array_equal(u.cpu().numpy(), u_host)
    y = torch.empty(rows, dtype=torch.float32, device="cuda")
    idx = np.concatenate([np.arange(4 * bi, 4 * bi + 4) for bi in SAMPLE_BR])
    M_s = np.concatenate([source_rows[bi] for bi in SAMPLE_BR])            # (4 * nsample, cols) FP32
    # the GPU generator's rows are the host generator's rows
    got_rows = dense[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.array_equal(got_rows.view(np.uint32), M_s.view(np.uint32))
    ref_src = M_s.astype(np.float64) @ u_host.astype(np.float64)
    tol = {wh.WH_FMT_F32: 1e-6, wh.WH_FMT_F16: 2e-3, wh.WH_FMT_BF16: 2e-3, wh.WH_FMT_FP8E4M3_BS4: 2e-2}
    nbc = cols // 4
    nb = NBR * nbc
    for fmt in (wh.WH_FMT_F32, wh.WH_FMT_F16, wh.WH_FMT_BF16, wh.WH_FMT_FP8E4M3_BS4):
        if fmt == wh.WH_FMT_F32:
            store = dense
        else:
            store = torch.empty(wh.wh_storage_bytes(rows, cols, fmt), dtype=torch.uint8, device="cuda")
            wh.wh_quantize(gpu_ctx, dense, fmt, store)
        mat = wh.wh_load_compressed(gpu_ctx, rows, cols, fmt, 0, store)
        wh.wh_gemv(gpu_ctx, mat, u, y, 0, rows)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        # codes on the sampled rows, and the oracle's dequantised rows
        if fmt == wh.WH_FMT_F32:
            deq = M_s.astype(np.float64)
        elif fmt in (wh.WH_FMT_F16, wh.WH_FMT_BF16):
            st16 = store.view(torch.int16).view(rows, cols)[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.uint16)
            if fmt == wh.WH_FMT_F16:
                want = quant.to_f16(M_s).view(np.uint16)
                deq = quant.to_f16(M_s).astype(np.float64)
            else:
                want = quant.bf16_bits(M_s)
                deq = quant.bf16_values(want).astype(np.float64)
            assert np.array_equal(st16, want), f"fmt {fmt}: codes differ on the sampled rows"
        else:
            deq_rows = []
            for bi in SAMPLE_BR:
                codes, scales = quant.fp8_block_scaled(source_rows[bi])
                c_gpu = store[bi * nbc * 16:(bi + 1) * nbc * 16].cpu().numpy().reshape(nbc, 16)
                s_gpu = store[nb * 16 + bi * nbc * 4: nb * 16 + (bi + 1) * nbc * 4].cpu().numpy().view(np.float32)
                assert np.array_equal(c_gpu, codes), f"FP8 codes differ at block row {bi}"
                assert np.array_equal(s_gpu.view(np.uint32), scales.view(np.uint32)), f"FP8 scales differ at {bi}"
                deq_rows.append(quant.fp8_dequant(codes, scales, 4, cols))
            deq = np.concatenate(deq_rows)
        e_src = rel_l2(yh[idx], ref_src)
        e_q = rel_l2(yh[idx], deq @ u_host.astype(np.float64))
        print(f"65536^2 dense fmt {fmt}: sampled rel-L2 vs FP32 source {e_src:.3e} (tol {tol[fmt]}), "
              f"vs dequantised {e_q:.3e}")
        assert e_src <= tol[fmt]
        assert e_q <= 1e-6
        assert np.all(np.isfinite(yh))
        wh.wh_unload(gpu_ctx, mat)
        if fmt != wh.WH_FMT_F32:
            del store
    del dense
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def large_rate8(gpu_ctx, source_rows):
    stream = workload.build_stream(gpu_ctx, SPEC, 8)
    mat = wh.wh_load_compressed(gpu_ctx, SPEC.rows, SPEC.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, stream)
    per = wh.stream_bytes(4, SPEC.cols, 8)
    decoded = {}
    for bi in SAMPLE_BR:
        s_ref = oracle.encode(source_rows[bi], 8)
        assert np.array_equal(stream[bi * per:(bi + 1) * per].cpu().numpy(), s_ref), bi
        decoded[bi] = oracle.decode(s_ref, 4, SPEC.cols, 8).astype(np.float64)
    yield mat, decoded
    wh.wh_unload(gpu_ctx, mat)
    del stream
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [4, 16, 64])
@pytest.mark.parametrize("udt", ["f32", "bf16"])
def test_multi_rhs_full_size(gpu_ctx, large_rate8, k, udt):
    mat, decoded = large_rate8
    U = synth.u_batch(SPEC, k)
    Ut = torch.from_numpy(U)
    if udt == "bf16":
        Ut = Ut.to(torch.bfloat16)
    U64 = Ut.float().numpy().astype(np.float64)
    Y = torch.empty((k, SPEC.rows), dtype=torch.float32, device="cuda")
    wh.wh_gemv_batched(gpu_ctx, mat, Ut.cuda(), Y)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(4 * bi, 4 * bi + 4) for bi in SAMPLE_BR])
    Yh = Y[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    Mhat = np.concatenate([decoded[bi] for bi in SAMPLE_BR])
    ref = U64 @ Mhat.T
    err = np.linalg.norm(Yh - ref, axis=1) / np.linalg.norm(ref, axis=1)
    tol = 1e-6 if udt == "f32" else 2e-3
    print(f"65536^2 rate 8 multi-RHS k={k} {udt}: worst per-RHS sampled rel-L2 {err.max():.3e} (tol {tol})")
    assert err.max() <= tol
    assert bool(torch.isfinite(Y).all())
