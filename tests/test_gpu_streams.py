"""Calls on different streams share the context's FP64 slab-partials
workspace (every plan that splits the columns uses it).  The library orders
such calls on the device, whatever stream they come on: queued back to back
on two streams with no host synchronisation, each result still matches the
FP64 oracle within 1e-6 relative L2, and repeats are bit-identical.
Covered: the fused compressed GEMV, dense FP32, the multi-RHS kernel and the
host-resident pipeline, interleaved.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1902_08018_amd import synth, wh

pytestmark = pytest.mark.gpu

SHAPES = [(2048, 8192, 61), (1032, 4100, 62)]  # rows, cols, seed


def rel_l2(y, ref):
    y = np.asarray(y, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def test_two_streams_share_the_partials(gpu_ctx):
    for rows, cols, _ in SHAPES:  # both plans split the columns: the workspace is in use
        assert wh.wh_gemv_plan_info(rows, cols)["nslab"] > 1
    codes, mats, us, u_np, refs = [], [], [], [], []
    for rows, cols, seed in SHAPES:
        s = oracle.encode(synth.matrix(synth.MatrixSpec(rows, cols, 32, 8.0, seed=seed)), 8)
        d = torch.from_numpy(s).cuda()
        codes.append((s, d))
        mats.append(wh.wh_load_compressed(gpu_ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, d))
        u = synth.uniform(cols, seed=seed + 100)
        u_np.append(u)
        us.append(torch.from_numpy(u).cuda())
        refs.append(oracle.gemv_fp64(s, rows, cols, 8, u))
    (r0, c0, _), (r1, c1, _) = SHAPES
    # dense FP32 of the first matrix's source
    M0 = synth.matrix(synth.MatrixSpec(r0, c0, 32, 8.0, seed=SHAPES[0][2]))
    M0d = torch.from_numpy(M0).cuda()
    dmat = wh.wh_load_compressed(gpu_ctx, r0, c0, wh.WH_FMT_F32, 0, M0d)
    ref_d = M0.astype(np.float64) @ u_np[0].astype(np.float64)
    # multi-RHS on the first compressed matrix
    U = torch.from_numpy(synth.uniform(5 * c0, seed=300).reshape(5, c0)).cuda()
    ref_U = U.cpu().numpy().astype(np.float64) @ oracle.decode(codes[0][0], r0, c0, 8).astype(np.float64).T
    # the second compressed matrix also from page-locked host memory
    h1 = torch.empty(codes[1][0].size, dtype=torch.uint8, pin_memory=True)
    h1.copy_(torch.from_numpy(codes[1][0]))

    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    reps = 4
    y0 = [torch.full((r0,), -7.0, device="cuda") for _ in range(reps)]
    y1 = [torch.full((r1,), -7.0, device="cuda") for _ in range(reps)]
    yd = [torch.full((r0,), -7.0, device="cuda") for _ in range(reps)]
    yU = [torch.full((5, r0), -7.0, device="cuda") for _ in range(reps)]
    yh = [torch.full((r1,), -7.0, device="cuda") for _ in range(reps)]
    torch.cuda.synchronize()
    for rep in range(reps):
        a, b = streams[rep % 2], streams[(rep + 1) % 2]
        wh.wh_gemv(gpu_ctx, mats[0], us[0], y0[rep], 0, r0, stream=a)
        wh.wh_gemv(gpu_ctx, mats[1], us[1], y1[rep], 0, r1, stream=b)
        wh.wh_gemv_batched(gpu_ctx, mats[0], U, yU[rep], stream=a)
        wh.wh_gemv(gpu_ctx, dmat, us[0], yd[rep], 0, r0, stream=b)
        wh.wh_gemv_host(gpu_ctx, h1, r1, c1, 8, us[1], yh[rep], chunk_rows=64, stream=a)
    torch.cuda.synchronize()
    for ys, ref in ((y0, refs[0]), (y1, refs[1]), (yh, refs[1]), (yd, ref_d)):
        first = ys[0].cpu().numpy()
        assert rel_l2(first, ref) <= 1e-6
        for rep in range(1, reps):
            assert np.array_equal(ys[rep].cpu().numpy().view(np.uint32), first.view(np.uint32)), rep
    for rep in range(reps):
        Y = yU[rep].cpu().numpy().astype(np.float64)
        err = np.linalg.norm(Y - ref_U, axis=1) / np.linalg.norm(ref_U, axis=1)
        assert err.max() <= 1e-6, rep
    for m in mats + [dmat]:
        wh.wh_unload(gpu_ctx, m)
