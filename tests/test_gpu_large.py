"""Parity at the full 65536 x 65536 size, in the launch configuration the
benchmark times (whole matrix resident, one wh_gemv over all rows).

The oracle cannot decode 2^28 blocks in seconds, so it checks sampled
block-rows: it generates those rows of M on the host, encodes them itself,
and (1) the GPU-built stream must hold exactly the oracle's bytes there,
(2) the GPU y on those rows must be within relative L2 1e-6 of the oracle's
FP64 product, (3) the whole-matrix decode into row-major FP32 (the
separate path's first step, whose launch walks its 8 x 8 block patches in
a grid-stride loop at this size) must hold exactly the oracle's decoded
values on those rows.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1902_08018_amd import synth, wh, workload

pytestmark = pytest.mark.gpu

SAMPLE_ROWS = [0, 4, 16380, 32768, 40000, 65532]  # first row of each sampled block-row


@pytest.mark.parametrize("rate", [8, 16])
def test_large_config_sampled_rows(gpu_ctx, rate):
    spec = synth.LARGE
    stream = workload.build_stream(gpu_ctx, spec, rate)
    mat = wh.wh_load_compressed(gpu_ctx, spec.rows, spec.cols, wh.WH_FMT_ZFP_FIXED_RATE, rate, stream)
    u = workload.u_device(spec)
    y = torch.empty(spec.rows, dtype=torch.float32, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, u, y, 0, spec.rows)
    torch.cuda.synchronize()
    y_host = y.cpu().numpy()
    u_host = synth.u_vector(spec)
    assert np.array_equal(u.cpu().numpy(), u_host)
    table = synth.kernel_table(spec)
    per_brow = oracle.stream_nbytes(4, spec.cols, rate)
    errs = []
    got_all, ref_all, s_refs = [], [], []
    for r0 in SAMPLE_ROWS:
        M = synth.matrix_rows(spec, r0, r0 + 4, table)
        s_ref = oracle.encode(M, rate)
        s_refs.append(s_ref)
        bi = r0 // 4
        s_gpu = stream[bi * per_brow:(bi + 1) * per_brow].cpu().numpy()
        assert np.array_equal(s_gpu, s_ref), f"stream bytes differ at block-row {bi}"
        ref = oracle.gemv_fp64(s_ref, 4, spec.cols, rate, u_host)
        got_all.append(y_host[r0:r0 + 4])
        ref_all.append(ref)
        errs.append(np.abs(y_host[r0:r0 + 4] - ref).max() / np.abs(ref).max())
    got_all, ref_all = np.concatenate(got_all), np.concatenate(ref_all)
    err = float(np.linalg.norm(got_all - ref_all) / np.linalg.norm(ref_all))
    print(f"65536^2 rate {rate}: sampled rel-L2 {err:.3e}, worst row rel {max(errs):.3e}")
    assert err <= 1e-6
    # every row of y is finite and positive (M > 0 almost everywhere, u >= 0)
    assert np.all(np.isfinite(y_host))
    dense = torch.empty((spec.rows, spec.cols), dtype=torch.float32, device="cuda")
    wh.wh_decode(gpu_ctx, mat, dense)
    torch.cuda.synchronize()
    for r0, s_ref in zip(SAMPLE_ROWS, s_refs):
        got = dense[r0:r0 + 4].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), oracle.decode(s_ref, 4, spec.cols, rate).view(np.uint32)), r0
    del dense
    wh.wh_unload(gpu_ctx, mat)
    del stream
    torch.cuda.empty_cache()
