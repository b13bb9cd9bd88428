"""GPU parity of wh_gemv_host: a WHZ1 matrix that stays in host memory,
its block rows streamed over the link in chunks while the fused kernel works
on the chunk before (Sec. 4.2-4.3, Table 1).

  y against the FP64 oracle within 1e-6 relative L2 (Fig. 7 mode: within 1
  FP32 ulp), for chunk sizes from one block row up, row ranges that start
  and end inside block rows, page-locked and pageable host memory; the
  direct mode (the kernel reads page-locked host memory itself); calls in a
  row on two streams that share the staging buffers; argument errors.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1902_08018_amd import synth, wh, workload

pytestmark = pytest.mark.gpu


def rel_l2(y, ref):
    y = np.asarray(y, dtype=np.float64)
    return float(np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300))


def case(rows, cols, rate=8, seed=41):
    spec = synth.MatrixSpec(rows, cols, 32, 8.0, seed=seed)
    return oracle.encode(synth.matrix(spec), rate)


def pinned(s):
    t = torch.empty(s.size, dtype=torch.uint8, pin_memory=True)
    t.copy_(torch.from_numpy(s))
    return t


@pytest.mark.parametrize("rows,cols", [(378, 262), (1030, 1030), (61, 4096), (5, 7)])
@pytest.mark.parametrize("chunk_rows", [0, 4, 12, 64])
def test_host_stream_matches_oracle(gpu_ctx, rows, cols, chunk_rows):
    s = case(rows, cols)
    h = pinned(s)
    u_np = synth.uniform(cols, seed=11)
    u = torch.from_numpy(u_np).cuda()
    ref = oracle.gemv_fp64(s, rows, cols, 8, u_np)
    for rb, re in [(0, rows), (3, rows - 2), (rows - 5, rows), (1, 2)]:
        if not 0 <= rb < re <= rows:
            continue
        y = torch.full((re - rb + 2,), -7.0, device="cuda")
        wh.wh_gemv_host(gpu_ctx, h, rows, cols, 8, u, y, rb, re, chunk_rows)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        assert rel_l2(yh[:re - rb], ref[rb:re]) <= 1e-6, (rb, re)
        assert np.all(yh[re - rb:] == -7.0)


def test_host_stream_library_pinned_buffer(gpu_ctx):
    rows, cols = 262, 2050
    s = case(rows, cols, seed=44)
    hb = wh.HostBuffer(s.size)
    try:
        hb.array[:] = s
        u_np = synth.uniform(cols, seed=14)
        y = torch.empty(rows, device="cuda")
        wh.wh_gemv_host(gpu_ctx, hb.array, rows, cols, 8, torch.from_numpy(u_np).cuda(), y, chunk_rows=32)
        torch.cuda.synchronize()
        assert rel_l2(y.cpu().numpy(), oracle.gemv_fp64(s, rows, cols, 8, u_np)) <= 1e-6
    finally:
        hb.close()


@pytest.mark.parametrize("rows,cols", [(378, 262), (1030, 1030), (5, 7)])
def test_host_direct_matches_oracle(gpu_ctx, rows, cols):
    """WH_HOST_DIRECT: the fused kernel reads the page-locked stream itself."""
    s = case(rows, cols, seed=45)
    h = pinned(s)
    u_np = synth.uniform(cols, seed=15)
    u = torch.from_numpy(u_np).cuda()
    ref = oracle.gemv_fp64(s, rows, cols, 8, u_np)
    for rb, re in [(0, rows), (3, rows - 2), (1, 2)]:
        if not 0 <= rb < re <= rows:
            continue
        y = torch.full((re - rb + 2,), -7.0, device="cuda")
        wh.wh_gemv_host(gpu_ctx, h, rows, cols, 8, u, y, rb, re, flags=wh.WH_HOST_DIRECT)
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        assert rel_l2(yh[:re - rb], ref[rb:re]) <= 1e-6, (rb, re)
        assert np.all(yh[re - rb:] == -7.0)


def test_host_stream_pageable_and_modes(gpu_ctx):
    rows, cols = 130, 1030
    s = case(rows, cols, rate=16)
    u_np = synth.uniform(cols, seed=12)
    u = torch.from_numpy(u_np).cuda()
    ref = oracle.gemv_fp64(s, rows, cols, 16, u_np)
    y = torch.empty(rows, device="cuda")
    wh.wh_gemv_host(gpu_ctx, s, rows, cols, 16, u, y, chunk_rows=8)  # pageable numpy memory
    torch.cuda.synchronize()
    assert rel_l2(y.cpu().numpy(), ref) <= 1e-6
    wh.wh_gemv_host(gpu_ctx, s, rows, cols, 16, u, y, chunk_rows=8, flags=wh.WH_ACC_TWOSUM)
    torch.cuda.synchronize()
    assert rel_l2(y.cpu().numpy(), ref) <= 1e-6
    ref_mp = oracle.gemv_paper_mp(s, rows, cols, 16, u_np).astype(np.float64)
    wh.wh_gemv_host(gpu_ctx, s, rows, cols, 16, u, y, chunk_rows=8, flags=wh.WH_PAPER_MP)
    torch.cuda.synchronize()
    g = y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(g - ref_mp) <= np.spacing(np.abs(ref_mp).astype(np.float32)))


def test_host_stream_calls_in_a_row_on_two_streams(gpu_ctx):
    """Calls queued back to back on two streams, with no synchronisation
    between them, share the staging buffers: each still gets its own y."""
    mats = [(262, 2050, 51), (1030, 1030, 52), (64, 4096, 53)]
    hs, refs, us, ys = [], [], [], []
    for rows, cols, seed in mats:
        s = case(rows, cols, seed=seed)
        u_np = synth.uniform(cols, seed=seed)
        hs.append(pinned(s))
        refs.append(oracle.gemv_fp64(s, rows, cols, 8, u_np))
        us.append(torch.from_numpy(u_np).cuda())
        ys.append(torch.empty(rows, device="cuda"))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(3):
        for i, (rows, cols, _) in enumerate(mats):
            wh.wh_gemv_host(gpu_ctx, hs[i], rows, cols, 8, us[i], ys[i], chunk_rows=16,
                            stream=streams[(i + rep) % 2])
    torch.cuda.synchronize()
    for i in range(len(mats)):
        assert rel_l2(ys[i].cpu().numpy(), refs[i]) <= 1e-6, i


def test_host_stream_field_slit(gpu_ctx):
    """The paper's flow at its shapes: the 2116 x 256000 field matrix (rate 8)
    in page-locked host memory, a 378-row slit window and the whole field,
    against the oracle on the window and the resident-matrix GEMV on the
    field."""
    rows, cols = 2116, 256000
    spec = synth.MatrixSpec(rows, cols, 512, 32.0, seed=4)
    st = workload.build_stream(gpu_ctx, spec, 8)
    h = torch.empty(st.numel(), dtype=torch.uint8, pin_memory=True)
    h.copy_(st)
    s = h.numpy()
    u_np = synth.uniform(cols, seed=13)
    u = torch.from_numpy(u_np).cuda()
    y = torch.empty(378, device="cuda")
    wh.wh_gemv_host(gpu_ctx, h, rows, cols, 8, u, y, 1001, 1379)
    torch.cuda.synchronize()
    ref = oracle.gemv_fp64(s, rows, cols, 8, u_np, row_begin=1001, row_end=1379, nthreads=8)
    assert rel_l2(y.cpu().numpy(), ref) <= 1e-6
    mat = wh.wh_load_compressed(gpu_ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, st)
    yr = torch.empty(rows, device="cuda")
    wh.wh_gemv(gpu_ctx, mat, u, yr, 0, rows)
    yf = torch.empty(rows, device="cuda")
    wh.wh_gemv_host(gpu_ctx, h, rows, cols, 8, u, yf)
    torch.cuda.synchronize()
    a, b = yf.cpu().numpy().astype(np.float64), yr.cpu().numpy().astype(np.float64)
    assert float(np.linalg.norm(a - b) / np.linalg.norm(b)) <= 2e-6
    wh.wh_unload(gpu_ctx, mat)


def test_host_stream_argument_errors(gpu_ctx):
    rows, cols = 16, 32
    s = case(rows, cols)
    u = torch.rand(cols, device="cuda")
    y = torch.empty(32, device="cuda")
    for kw, code in [(dict(chunk_rows=6), wh.WH_ERR_INVALID), (dict(row_begin=0, row_end=17), wh.WH_ERR_SHAPE),
                     (dict(row_begin=9, row_end=8), wh.WH_ERR_SHAPE), (dict(flags=3), wh.WH_ERR_INVALID)]:
        with pytest.raises(wh.WhError) as ei:
            wh.wh_gemv_host(gpu_ctx, s, rows, cols, 8, u, y, **kw)
        assert ei.value.status == code, kw
    with pytest.raises(wh.WhError) as ei:
        wh.wh_gemv_host(gpu_ctx, np.zeros(4096, np.uint8), rows, cols, 7, u, y)
    assert ei.value.status == wh.WH_ERR_FORMAT
    with pytest.raises(ValueError):
        wh.wh_gemv_host(gpu_ctx, s[:-1], rows, cols, 8, u, y)
    wh.wh_gemv_host(gpu_ctx, s, rows, cols, 8, u, y, 5, 5)  # empty range: no-op
