"""GPU parity of the multi-right-hand-side path (decode -> LDS -> MFMA).

Reference: the oracle-decoded matrix in FP64 times the k vectors (a plain
FP64 matrix product of the oracle's decode).  Bounds: FP32 vectors, relative
L2 1e-6 per right-hand side, whether they run on the FP32 matrix cores
(4x4x1 MFMAs up to 4 right-hand sides, 16x16x4 up to 16, or 16x16x4 always
with WH_MRHS_FP32=1) or split into three BF16 parts on the BF16 matrix cores
(from 17 up); BF16 vectors (the decoded values rounded to BF16 for the
contraction), 2e-3.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1902_08018_amd import synth, wh

pytestmark = pytest.mark.gpu


def per_rhs_rel_l2(Y, ref):
    Y = np.asarray(Y, dtype=np.float64)
    return np.linalg.norm(Y - ref, axis=1) / np.linalg.norm(ref, axis=1)


@pytest.fixture(scope="module")
def small_mrhs():
    M = synth.matrix(synth.SMALL)
    s = oracle.encode(M, 8)
    Mhat = oracle.decode(s, 4096, 4096, 8).astype(np.float64)
    return s, Mhat


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 9, 16, 17, 33, 64])
def test_mrhs_fp32(gpu_ctx, small_mrhs, k):
    s, Mhat = small_mrhs
    U = synth.u_batch(synth.SMALL, k)
    ref = U.astype(np.float64) @ Mhat.T          # (k, rows)
    d = torch.from_numpy(s).cuda()
    mat = wh.wh_load_compressed(gpu_ctx, 4096, 4096, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
    Y = torch.empty((k, 4096), dtype=torch.float32, device="cuda")
    wh.wh_gemv_batched(gpu_ctx, mat, torch.from_numpy(U).cuda(), Y)
    torch.cuda.synchronize()
    err = per_rhs_rel_l2(Y.cpu().numpy(), ref)
    print(f"k={k} FP32: worst per-RHS rel-L2 {err.max():.3e}")
    assert err.max() <= 1e-6
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("k", [4, 16, 20, 33, 64])  # every compiled width (16, 32, 48, 64 RHS)
def test_mrhs_bf16(gpu_ctx, small_mrhs, k):
    s, Mhat = small_mrhs
    U = synth.u_batch(synth.SMALL, k)
    Ub = torch.from_numpy(U).to(torch.bfloat16)
    ref = Ub.float().numpy().astype(np.float64) @ Mhat.T
    d = torch.from_numpy(s).cuda()
    mat = wh.wh_load_compressed(gpu_ctx, 4096, 4096, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
    Y = torch.empty((k, 4096), dtype=torch.float32, device="cuda")
    wh.wh_gemv_batched(gpu_ctx, mat, Ub.cuda(), Y)
    torch.cuda.synchronize()
    err = per_rhs_rel_l2(Y.cpu().numpy(), ref)
    print(f"k={k} BF16: worst per-RHS rel-L2 {err.max():.3e}")
    assert err.max() <= 2e-3
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("shape", [(4, 4), (68, 260), (260, 68), (1028, 1092)])
@pytest.mark.parametrize("rate", [8, 16])
@pytest.mark.parametrize("k", [3, 5, 40])
def test_mrhs_ragged(gpu_ctx, shape, rate, k):
    rows, cols = shape
    spec = synth.MatrixSpec(rows, cols, 32, 8.0, seed=13)
    M = synth.matrix(spec)
    s = oracle.encode(M, rate)
    Mhat = oracle.decode(s, rows, cols, rate).astype(np.float64)
    ldu, ldy = cols + 12, rows + 8  # padded leading dimensions
    Upad = np.zeros((k, ldu), dtype=np.float32)
    Upad[:, :cols] = synth.uniform(k * cols, seed=13).reshape(k, cols)
    ref = Upad[:, :cols].astype(np.float64) @ Mhat.T
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, rate, torch.from_numpy(s).cuda())
    Y = torch.full((k, ldy), -1.0, dtype=torch.float32, device="cuda")
    wh.wh_gemv_batched(gpu_ctx, mat, torch.from_numpy(Upad).cuda(), Y)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy()
    assert per_rhs_rel_l2(Yh[:, :rows], ref).max() <= 1e-6
    assert np.all(Yh[:, rows:] == -1.0)  # padding untouched
    wh.wh_unload(gpu_ctx, mat)


def test_mrhs_matches_single_vector_path(gpu_ctx, small_mrhs):
    """Each right-hand side of a batch equals (within the bound) the k = 1
    fused kernel's result for that vector alone."""
    s, _ = small_mrhs
    U = synth.u_batch(synth.SMALL, 8)
    d = torch.from_numpy(s).cuda()
    mat = wh.wh_load_compressed(gpu_ctx, 4096, 4096, wh.WH_FMT_ZFP_FIXED_RATE, 8, d)
    Ud = torch.from_numpy(U).cuda()
    Y = torch.empty((8, 4096), dtype=torch.float32, device="cuda")
    wh.wh_gemv_batched(gpu_ctx, mat, Ud, Y)
    y1 = torch.empty(4096, dtype=torch.float32, device="cuda")
    for j in range(8):
        wh.wh_gemv(gpu_ctx, mat, Ud[j].contiguous(), y1, 0, 4096)
        torch.cuda.synchronize()
        a, b = Y[j].cpu().numpy().astype(np.float64), y1.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 2e-6
    wh.wh_unload(gpu_ctx, mat)


def test_mrhs_argument_errors(gpu_ctx, small_mrhs):
    s, _ = small_mrhs
    mat = wh.wh_load_compressed(gpu_ctx, 4096, 4096, wh.WH_FMT_ZFP_FIXED_RATE, 8, torch.from_numpy(s).cuda())
    Y = torch.empty((65, 4096), dtype=torch.float32, device="cuda")
    with pytest.raises(wh.WhError) as ei:
        wh.wh_gemv_batched(gpu_ctx, mat, torch.zeros((65, 4096), device="cuda"), Y)
    assert ei.value.status == wh.WH_ERR_INVALID
    with pytest.raises(wh.WhError) as ei:
        wh.wh_gemv_batched(gpu_ctx, mat, torch.zeros((4, 4000), device="cuda"), Y[:4])
    assert ei.value.status == wh.WH_ERR_SHAPE
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("rate", [2, 4, 6])
@pytest.mark.parametrize("k", [3, 16, 40])
def test_mrhs_low_rates_wide_range(gpu_ctx, rate, k):
    """Rates where the bit budget cuts coefficients to their top planes,
    on wide-range data (rows scaled by 2^-30 .. 2^10, signs mixed): blocks
    cut above plane 26 take the exact inverse lift."""
    rng = np.random.default_rng(100 + rate)
    M = (rng.standard_normal((256, 1024)) * np.exp2(rng.integers(-30, 10, size=(256, 1)))).astype(np.float32)
    s = oracle.encode(M, rate)
    Mhat = oracle.decode(s, 256, 1024, rate).astype(np.float64)
    U = synth.uniform(k * 1024, seed=rate).reshape(k, 1024)
    ref = U.astype(np.float64) @ Mhat.T
    mat = wh.wh_load_compressed(gpu_ctx, 256, 1024, wh.WH_FMT_ZFP_FIXED_RATE, rate, s)
    Y = torch.empty((k, 256), dtype=torch.float32, device="cuda")
    wh.wh_gemv_batched(gpu_ctx, mat, torch.from_numpy(U).cuda(), Y)
    torch.cuda.synchronize()
    assert per_rhs_rel_l2(Y.cpu().numpy(), ref).max() <= 1e-6
    wh.wh_unload(gpu_ctx, mat)


@pytest.mark.parametrize("k", [3, 4, 17, 33, 64])
def test_mrhs_split_bf16_against_fp32_cores(small_mrhs, k):
    """Up to 4 right-hand sides FP32 vectors run on the 4x4x1 FP32 MFMA, from
    17 up as three BF16 parts on the BF16 matrix cores; a context made with
    WH_MRHS_FP32=1 keeps them on the 16x16x4 FP32 MFMA.  Both are within 1e-6
    of the oracle, and within 1e-6 of each other."""
    s, Mhat = small_mrhs
    U = synth.u_batch(synth.SMALL, k)
    ref = U.astype(np.float64) @ Mhat.T
    out = {}
    for force in (0, 1):
        old = os.environ.pop("WH_MRHS_FP32", None)
        if force:
            os.environ["WH_MRHS_FP32"] = "1"  # read by wh_create
        try:
            ctx = wh.wh_create(0, 0)
        finally:
            os.environ.pop("WH_MRHS_FP32", None)
            if old is not None:
                os.environ["WH_MRHS_FP32"] = old
        mat = wh.wh_load_compressed(ctx, 4096, 4096, wh.WH_FMT_ZFP_FIXED_RATE, 8, torch.from_numpy(s).cuda())
        Y = torch.empty((k, 4096), dtype=torch.float32, device="cuda")
        wh.wh_gemv_batched(ctx, mat, torch.from_numpy(U).cuda(), Y)
        torch.cuda.synchronize()
        out[force] = Y.cpu().numpy()
        wh.wh_destroy(ctx)
        err = per_rhs_rel_l2(out[force], ref)
        print(f"k={k} {'16x16x4 FP32' if force else 'default path'}: worst per-RHS rel-L2 {err.max():.3e}")
        assert err.max() <= 1e-6
    assert per_rhs_rel_l2(out[0], out[1].astype(np.float64)).max() <= 1e-6
