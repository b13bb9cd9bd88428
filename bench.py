#!/usr/bin/env python3
"""Benchmark: fused decode + mixed-precision GEMV over a zfp-compressed matrix.

Workload (the plain path at scale): M is 65536 x 65536 FP32 from
M[i,j] = exp(-|p_i - q_j| / 32) + N(0, 1e-4) on two 256 x 256 unit lattices,
held resident in HBM as a WHZ1 fixed-rate stream (8 bits/value: 4.29 GB);
u is 65536 values U[0,1).  One step = one wh_gemv over all rows (decode of
every block, FP32 block MAC, FP64 row accumulation, FP32 y).  Inputs are
resident before timing starts; 4 different u vectors rotate across steps.

Prints one JSON line.  `value` is the effective bandwidth in the paper's
decoder convention (uncompressed FP32 bytes of M per second, Sec. 4.3);
`roofline` prices the kernel's algorithmic bytes (compressed stream + u + y)
against the 8 TB/s HBM peak, with the box's measured copy ceiling beside
it and, when a counter run on the same kernel source is on file, the VALU
issue roofline that actually bounds the decoder; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload on this host (all cores and
one core); `parity_vs_oracle` checks the timed configuration's first rows
against the oracle's FP64 GEMV.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
# VALU: the published FP32 vector rate (157.3 TFLOP/s, an FMA counting two)
# in lane operations: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz, T lane-ops/s.
# (The kernel's measured issue rate, 628 G wave64 instructions/s, is above the
# 614 G/s that 16 lanes per SIMD per cycle would allow.)
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
PARITY_ROWS = 256


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rate", type=int, default=8)
    ap.add_argument("--size", type=int, default=65536, help="rows = cols (256x256 lattices at 65536)")
    ap.add_argument("--flags", type=int, default=0, help="wh_gemv flags (0 default, 1 FP64, 2 TwoSum, 4 Fig. 7)")
    ap.add_argument("--extra", type=int, default=1, help="also time rate 16 and the separate path")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--serving", type=int, default=1, help="also run the Poisson serving load")
    ap.add_argument("--serving-requests", type=int, default=20000)
    ap.add_argument("--leg", default="", help="'host-pipeline' (internal), 'serving' (the three-matrix load of "
                                              "--serving-requests requests), 'thermal' (the thermal step) or "
                                              "'var' (the variable-rate modes on a --var-size square matrix) runs "
                                              "only that leg and prints its JSON")
    ap.add_argument("--var-size", type=int, default=8192, help="matrix side of --leg var")
    ap.add_argument("--probe", type=int, default=0,
                    help="counter-pass mode, prints no JSON: 1 = 3 launches of the timed configuration, then 3 "
                         "plain 4 GiB device copies (the calibration kernel for FETCH_SIZE / WRITE_SIZE) and 3 "
                         "read-only streams of the same 4 GiB; "
                         "2 = 3 multi-RHS launches (k = --probe-k, FP32 or --probe-bf16 U) on the same matrix; "
                         "3 = 3 whole-matrix decodes into row-major FP32 (the separate path's first step)")
    ap.add_argument("--probe-k", type=int, default=16, help="right-hand sides of --probe 2")
    ap.add_argument("--probe-bf16", type=int, default=0, help="--probe 2 with BF16 U")
    ap.add_argument("--traffic-json", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                                           "traffic.json"))
    return ap.parse_args()


def kernel_source_hash() -> str:
    """Hash of the fused kernel's source (decoder header + kernels)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1902_08018_amd", "csrc")
    for name in ("whz_device.hpp", "whz_kernels.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def time_gemv(ctx, mat, us, y, rows, steps, warmup, flags):
    """Event-timed wh_gemv launches on torch's current stream (the stream the
    library launches on).  Returns (wall ms/step, per-launch event ms list)."""
    import torch
    from paper_1902_08018_amd import wh
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        wh.wh_gemv(ctx, mat, us[i % len(us)], y, 0, rows, flags)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        wh.wh_gemv(ctx, mat, us[i % len(us)], y, 0, rows, flags)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    return wall_ms, [a.elapsed_time(b) for a, b in ev]


def time_call(fn, steps, warmup):
    """Mean event-timed ms of fn() on torch's current stream (the stream the
    library launches on when none is given)."""
    import torch
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        fn(i)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


class SampledRows:
    """Oracle references for sampled block rows of a synthetic matrix, so that
    every timed result carries its error: the host generator makes those rows
    of the FP32 source, the oracle encodes them itself at the rate asked for
    and decodes them, and the references are FP64 products (numpy) of the
    source or of the oracle-decoded rows.  `brows` are block-row indices; a
    partial last block row is taken whole (its real rows only)."""

    def __init__(self, spec, nsample=16, brows=None):
        import numpy as np
        from paper_1902_08018_amd import synth
        self.spec = spec
        nbr = (spec.rows + 3) // 4
        if brows is None:
            brows = sorted(set([0, nbr - 1] + [int(x) for x in np.linspace(0, nbr - 1, nsample)]))
        self.brows = [b for b in brows if 0 <= b < nbr]
        table = synth.kernel_table(spec)
        self.src = [synth.matrix_rows(spec, 4 * b, min(4 * b + 4, spec.rows), table) for b in self.brows]
        self.idx = np.concatenate([np.arange(4 * b, 4 * b + m.shape[0]) for b, m in zip(self.brows, self.src)])
        self._dec = {}

    def source(self):
        import numpy as np
        return np.concatenate(self.src).astype(np.float64)

    def decoded(self, rate):
        """FP64 rows of the oracle's own fixed-rate encode + decode."""
        import numpy as np
        import oracle
        if rate not in self._dec:
            self._dec[rate] = np.concatenate([oracle.decode(oracle.encode(m, rate), m.shape[0], m.shape[1], rate)
                                              for m in self.src]).astype(np.float64)
        return self._dec[rate]

    def decoded_var(self, mode, param):
        import numpy as np
        import oracle
        key = ("var", mode, param)
        if key not in self._dec:
            out = []
            for m in self.src:
                code, index, _ = oracle.encode_var(m, mode, param)
                out.append(oracle.decode_var(code, index, m.shape[0], m.shape[1], mode, param))
            self._dec[key] = np.concatenate(out).astype(np.float64)
        return self._dec[key]

    def take(self, y, row0=0):
        """y's values at the sampled rows (y holds rows row0, row0 + 1, ...;
        a torch tensor (k, n) or (n,), or numpy)."""
        import numpy as np
        import torch
        sel = self.idx - row0
        if isinstance(y, torch.Tensor):
            t = torch.from_numpy(sel).to(y.device)
            return (y.index_select(y.dim() - 1, t)).cpu().numpy().astype(np.float64)
        return np.asarray(y, np.float64)[..., sel]


def err_entry(got, ref, tol):
    """Relative L2 (worst over right-hand sides for 2-D results) of the
    sampled rows against the oracle, with the bound it must meet."""
    import numpy as np
    got = np.atleast_2d(np.asarray(got, np.float64))
    ref = np.atleast_2d(np.asarray(ref, np.float64))
    e = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return {"rel_l2": float(f"{float(e.max()):.4g}"), "tolerance": tol, "ok": bool(e.max() <= tol)}


PRECISION_TOL = {"f32": 1e-6, "f16": 2e-3, "bf16": 2e-3, "fp8e4m3_bs4": 2e-2}


def bench_precision(ctx, spec, us, y, steps, sample):
    """Dense storage formats of the same FP32 matrix (no compression): FP32,
    FP16, BF16 and FP8 e4m3 with one FP32 scale per 4x4 block.  Each result's
    error: sampled rows of y for us[0] against the FP64 product of the FP32
    source rows."""
    import numpy as np
    import torch
    from paper_1902_08018_amd import synth, wh, workload
    rows, cols = spec.rows, spec.cols
    dense = workload.build_dense(spec)
    ref = sample.source() @ synth.u_vector(spec).astype(np.float64)
    res = {}
    for name, fmt in (("f32", wh.WH_FMT_F32), ("f16", wh.WH_FMT_F16), ("bf16", wh.WH_FMT_BF16),
                      ("fp8e4m3_bs4", wh.WH_FMT_FP8E4M3_BS4)):
        nbytes = wh.wh_storage_bytes(rows, cols, fmt)
        if fmt == wh.WH_FMT_F32:
            store = dense
        else:
            store = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            wh.wh_quantize(ctx, dense, fmt, store)
        m = wh.wh_load_compressed(ctx, rows, cols, fmt, 0, store)
        ms = time_call(lambda i: wh.wh_gemv(ctx, m, us[i % len(us)], y, 0, rows), steps, 2)
        wh.wh_gemv(ctx, m, us[0], y, 0, rows)
        alg = nbytes + 4 * cols + 4 * rows
        res[name] = {"ms": round(ms, 4), "storage_gb": round(nbytes / 1e9, 3),
                     "hbm_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "effective_gbs": round(4.0 * rows * cols / (ms * 1e-3) / 1e9, 1),
                     "error_vs_fp32_source": err_entry(sample.take(y), ref, PRECISION_TOL[name])}
        wh.wh_unload(ctx, m)
        if fmt != wh.WH_FMT_F32:
            del store
    del dense
    return res


def bench_multi_rhs(ctx, mat, spec, rate, stream_bytes, steps, sample):
    """k right-hand sides against the resident rate-`rate` stream (decode ->
    LDS -> matrix cores), FP32 and BF16 vectors.  Each result's error: sampled
    rows of Y against the FP64 product of the oracle-decoded rows with U (U
    rounded to BF16 for the BF16 leg), worst right-hand side."""
    import numpy as np
    import torch
    from paper_1902_08018_amd import synth, wh
    rows, cols = spec.rows, spec.cols
    Mhat = sample.decoded(rate)
    res = {}
    for k in (4, 16, 64):
        U32 = torch.from_numpy(synth.u_batch(spec, k)).cuda()
        Y = torch.empty((k, rows), dtype=torch.float32, device="cuda")
        for name, U in (("f32", U32), ("bf16", U32.to(torch.bfloat16))):
            ms = time_call(lambda i: wh.wh_gemv_batched(ctx, mat, U, Y), steps, 2)
            alg = stream_bytes + U.numel() * U.element_size() + Y.numel() * 4
            ref = U.float().cpu().numpy().astype(np.float64) @ Mhat.T
            res[f"k{k}_{name}"] = {"ms": round(ms, 4), "gflops": round(k * rows * (2 * cols - 1) / (ms * 1e-3) / 1e9, 1),
                                   "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                   "ms_per_rhs": round(ms / k, 4),
                                   "error_vs_oracle": err_entry(sample.take(Y), ref, 1e-6 if name == "f32" else 2e-3)}
    return res


# The paper's GEMV shapes (Sec. 5, Fig. 10): the slit matrix, its transpose
# and a square one; and a field matrix (about 2067 MB of FP32, Sec. 2.1) whose
# 378-row slit windows are multiplied one after another as the slit moves.
SLIT_SHAPES = (("wide_378x256000", 378, 256000), ("tall_256000x378", 256000, 378),
               ("square_10000x10000", 10000, 10000))
FIELD_ROWS, FIELD_COLS, SLIT_ROWS = 2116, 256000, 378


def bench_slit_field(ctx, rate, steps):
    """Fused decode + GEMV on the paper's GEMV shapes at `rate` bits/value,
    beside the dense FP32 GEMV of the same matrix (rows padded to a multiple
    of 4, which dense storage needs); and slit windows of a field matrix."""
    import torch
    from paper_1902_08018_amd import synth, wh, workload
    import numpy as np
    res = {}
    for name, rows, cols in SLIT_SHAPES:
        spec = synth.MatrixSpec(rows, cols, 512, 32.0, seed=3)
        st = workload.build_stream(ctx, spec, rate)
        m = wh.wh_load_compressed(ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, rate, st)
        us = [workload.u_device(spec, offset=i * cols) for i in range(4)]
        y = torch.empty(rows, dtype=torch.float32, device="cuda")
        ms = time_call(lambda i: wh.wh_gemv(ctx, m, us[i % 4], y, 0, rows), steps, 3)
        wh.wh_gemv(ctx, m, us[0], y, 0, rows)
        sample = SampledRows(spec, nsample=8)
        u64 = synth.u_vector(spec).astype(np.float64)
        wh.wh_unload(ctx, m)
        del st
        flop = rows * (2 * cols - 1)  # Eq. 3's GEMV count
        entry = {"ms": round(ms, 4), "gflops": round(flop / (ms * 1e-3) / 1e9, 1),
                 "effective_gbs": round(4.0 * rows * cols / (ms * 1e-3) / 1e9, 1),
                 "error_vs_oracle": err_entry(sample.take(y), sample.decoded(rate) @ u64, 1e-6)}
        prow, pcol = (rows + 3) // 4 * 4, (cols + 3) // 4 * 4
        if pcol == cols:
            pspec = synth.MatrixSpec(prow, cols, 512, 32.0, seed=3)
            dense = workload.build_dense(pspec)
            md = wh.wh_load_compressed(ctx, prow, cols, wh.WH_FMT_F32, 0, dense)
            yd = torch.empty(prow, dtype=torch.float32, device="cuda")
            msd = time_call(lambda i: wh.wh_gemv(ctx, md, us[i % 4], yd, 0, prow), steps, 3)
            wh.wh_gemv(ctx, md, us[0], yd, 0, prow)
            psample = SampledRows(pspec, nsample=8)
            wh.wh_unload(ctx, md)
            del dense
            entry["dense_f32"] = {"ms": round(msd, 4), "gflops": round(flop / (msd * 1e-3) / 1e9, 1),
                                  "hbm_frac": round(4.0 * prow * cols / (msd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "error_vs_fp32_source": err_entry(psample.take(yd), psample.source() @ u64, 1e-6)}
        res[name] = entry
    spec = synth.MatrixSpec(FIELD_ROWS, FIELD_COLS, 512, 32.0, seed=4)
    st = workload.build_stream(ctx, spec, rate)
    m = wh.wh_load_compressed(ctx, FIELD_ROWS, FIELD_COLS, wh.WH_FMT_ZFP_FIXED_RATE, rate, st)
    u = workload.u_device(spec)
    y = torch.empty(SLIT_ROWS, dtype=torch.float32, device="cuda")
    nwin = FIELD_ROWS - SLIT_ROWS + 1
    starts = [(i * 7) % nwin for i in range(max(steps, 16))]  # the slit steps 7 rows at a time

    def slit(i):
        r0 = starts[i % len(starts)]
        wh.wh_gemv(ctx, m, u, y, r0, r0 + SLIT_ROWS)
    ms = time_call(slit, len(starts), 3)
    # the last window's y against the oracle, on the block rows inside it
    r0 = starts[(len(starts) - 1) % len(starts)]
    torch.cuda.synchronize()
    fsample = SampledRows(spec, brows=list(range((r0 + 3) // 4, (r0 + SLIT_ROWS) // 4, 8)))
    flop = SLIT_ROWS * (2 * FIELD_COLS - 1)
    res[f"field_{FIELD_ROWS}x{FIELD_COLS}_slit_{SLIT_ROWS}_rows"] = {
        "ms": round(ms, 4), "gflops": round(flop / (ms * 1e-3) / 1e9, 1),
        "effective_gbs": round(4.0 * SLIT_ROWS * FIELD_COLS / (ms * 1e-3) / 1e9, 1),
        "field_stream_gb": round(st.numel() / 1e9, 3), "window_starts": "0, 7, 14, ... (mod 1739)",
        "error_vs_oracle": dict(err_entry(fsample.take(y, row0=r0),
                                          fsample.decoded(rate) @ synth.u_vector(spec).astype(np.float64), 1e-6),
                                window=f"rows {r0}..{r0 + SLIT_ROWS}")}
    wh.wh_unload(ctx, m)
    del st
    res["rate"] = rate
    res["paper_context"] = "P100 mixed-precision GEMV, uncompressed: 198.3 / 65.9 / 202.6 GFLOP/s (wide / tall / square)"
    return res


def bench_host_pipeline(ctx, rate, steps, modes=("chunk_32MiB", "chunk_8MiB", "direct"), parts=True):
    """Table 1 measured: a compressed matrix kept in page-locked host memory
    and streamed over the link by wh_gemv_host, chunks of block rows copied
    while the fused kernel works on the chunk before (Sec. 4.2-4.3).  Beside
    it, the parts of Table 1's formulas measured on their own: the plain
    host-to-device copy of the same compressed bytes (T_transfer / R) and the
    fused kernel on the resident matrix (T_compute + T_decode).  The pipeline
    is timed first, before the device allocations of the parts."""
    import numpy as np
    import torch
    from paper_1902_08018_amd import synth, wh, workload
    res = {}
    for name, spec in (("field_2116x256000", synth.MatrixSpec(FIELD_ROWS, FIELD_COLS, 512, 32.0, seed=4)),
                       ("65536x65536", synth.LARGE)):
        print(f"# host pipeline: {name}", file=sys.stderr, flush=True)
        rows, cols = spec.rows, spec.cols
        st = workload.build_stream(ctx, spec, rate)
        h = torch.empty(st.numel(), dtype=torch.uint8, pin_memory=True)
        h.copy_(st)
        u = workload.u_device(spec)
        y = torch.empty(rows, dtype=torch.float32, device="cuda")
        entry = {"compressed_gb": round(h.numel() / 1e9, 3), "uncompressed_gb": round(4.0 * rows * cols / 1e9, 3),
                 "R": 32 / rate}
        sample = SampledRows(spec, nsample=8)
        ref = sample.decoded(rate) @ synth.u_vector(spec).astype(np.float64)
        chunk8 = 4 * max(1, (8 << 20) // wh.stream_bytes(4, cols, rate))
        # settle: half a second of calls before timing
        t_end = time.perf_counter() + 0.5
        while time.perf_counter() < t_end:
            wh.wh_gemv_host(ctx, h, rows, cols, rate, u, y)
            torch.cuda.synchronize()
        for chunk_rows, flags, label in ((0, 0, "chunk_32MiB"), (chunk8, 0, "chunk_8MiB"),
                                         (0, wh.WH_HOST_DIRECT, "direct")):
            if label not in modes:
                continue
            call = (lambda i: wh.wh_gemv_host(ctx, h, rows, cols, rate, u, y, 0, rows, chunk_rows, flags))
            period = time_call(call, 3, 2)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            lat = []
            for _ in range(3):  # from an idle device: the copy of the first chunk to the last y
                e0.record()
                call(0)
                e1.record()
                torch.cuda.synchronize()
                lat.append(e0.elapsed_time(e1))
            entry[label] = {"period_ms": round(period, 3), "latency_ms": round(min(lat), 3),
                            "effective_gbs": round(4.0 * rows * cols / (period * 1e-3) / 1e9, 1),
                            "error_vs_oracle": err_entry(sample.take(y), ref, 1e-6)}
        if not parts:
            res[name] = entry
            del h, st
            continue
        # the parts of Table 1
        m = wh.wh_load_compressed(ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, rate, st)
        t_fused = time_call(lambda i: wh.wh_gemv(ctx, m, u, y, 0, rows), steps, 2)
        wh.wh_unload(ctx, m)
        t_copy = time_call(lambda i: st.copy_(h, non_blocking=True), 3, 1)
        del st
        link_gbs = h.numel() / (t_copy * 1e-3) / 1e9
        entry.update({"link_h2d_gbs": round(link_gbs, 1), "t_copy_compressed_ms": round(t_copy, 3),
                      "t_fused_resident_ms": round(t_fused, 3)})
        # Table 1 with the measured parts (T_compute << T_transfer for a GEMV, Sec. 4.3)
        t_transfer = 4.0 * rows * cols / (link_gbs * 1e9) * 1e3
        entry["table1_ms"] = {"period_without_compression": round(t_transfer, 3),
                              "period_with": round(max(t_transfer / entry["R"], t_fused), 3),
                              "latency_with": round(t_fused + t_transfer / entry["R"], 3)}
        res[name] = entry
        del h
    return res


def host_pipeline_child(rate, steps):
    """The pipeline leg in a child process of its own, as a process that
    only streams a host-resident matrix would run it.  (In a process that has
    run the other legs first, the library's chunk copies were measured at
    about half the link rate, cause unresolved; that figure is reported
    beside this one.)"""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--leg", "host-pipeline", "--rate", str(rate),
           "--steps", str(steps), "--cpu-baseline", "0", "--serving", "0"]
    # the child's progress lines go to this process's stderr as they come
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": f"child exited {r.returncode}"}
    return json.loads(r.stdout.strip().splitlines()[-1])


def bench_thermal(ctx, steps):
    """The thermal step of Eq. 1 on the 608 x 608 mesh (369,664 temperatures,
    the paper's ~3.7e5), one launch per step: single steps back to back, and a
    100-step run.  Algorithmic bytes per step: the CSR (row pointers, 8 B per
    entry), b, u, T read once and T_next written."""
    import numpy as np
    import torch
    from paper_1902_08018_amd import synth, wh
    spec = synth.THERMAL
    row_ptr, col, val, b = synth.thermal_system(spec)
    dev = wh.ThermalSystem(row_ptr, col, val, b)
    n, nnz = spec.n, dev.nnz
    T = [torch.from_numpy(synth.thermal_initial(spec)).cuda(), torch.empty(n, device="cuda")]
    K = 100
    U = torch.from_numpy(np.stack([synth.thermal_source(spec, k) for k in range(K)])).cuda()
    one = time_call(lambda i: wh.wh_thermal_step(ctx, dev, T[i % 2], U[i % K], T[(i + 1) % 2]), max(steps, 50), 5)
    # one step from a known state against the oracle's FP64 step
    import oracle.thermal
    T0 = synth.thermal_initial(spec)
    T[0].copy_(torch.from_numpy(T0))
    wh.wh_thermal_step(ctx, dev, T[0], U[0], T[1])
    t1 = T[1].cpu().numpy()
    ref1 = oracle.thermal.thermal_step(row_ptr, col, val, b, T0, U[0].cpu().numpy())
    run = time_call(lambda i: wh.wh_thermal_run(ctx, dev, T[0], U, T[1]), 3, 1) / K
    alg = 4 * (n + 1) + 8 * nnz + 16 * n
    flop = 2 * nnz + n  # Eq. 3's thermal term: 2 nnz(A) + 2 nnz(B) - 1 per row
    res = {"n": n, "nnz": nnz, "bytes_per_step": alg, "error_vs_oracle": err_entry(t1, ref1, 1e-6)}
    for name, ms in (("single_step", one), ("run_100_steps_per_step", run)):
        res[name] = {"us": round(ms * 1e3, 2), "hbm_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "gflops": round(flop / (ms * 1e-3) / 1e9, 1)}
    return res


VAR_SPEC_ARGS = (8192, 8192, 128, 16.0)


def bench_var(ctx, steps):
    """The variable-rate modes (Sec. 4.3, Table 2) on an 8192 x 8192 synthetic
    matrix (VAR_SPEC_ARGS), beside fixed rate 8: bits per value (index included), the
    Table 2 error columns (NRMSE over the source's range, PSNR =
    -20 log10(2 NRMSE)), the host encoder's time, the GPU decode rate in the
    paper's W_c convention (uncompressed bytes per second) and the fused
    decode + GEMV."""
    import numpy as np
    import torch
    from paper_1902_08018_amd import synth, wh
    spec = synth.MatrixSpec(*VAR_SPEC_ARGS)
    rows, cols = spec.rows, spec.cols
    M = synth.matrix(spec)
    Md = torch.from_numpy(M).cuda()
    rng = float(M.max() - M.min())
    import oracle
    u = torch.from_numpy(synth.u_vector(spec)).cuda()
    u64 = synth.u_vector(spec).astype(np.float64)
    sample = SampledRows(spec, nsample=8)
    y = torch.empty(rows, device="cuda")
    out = torch.empty((rows, cols), device="cuda")
    res = {"matrix": f"{rows}x{cols}, 128-wide lattices, ell 16"}
    cases = [("fixed_rate_8", wh.WH_FMT_ZFP_FIXED_RATE, 8),
             ("fixed_precision_17", wh.WH_FMT_ZFP_FIXED_PRECISION, 17),
             ("fixed_accuracy_2^-20", wh.WH_FMT_ZFP_FIXED_ACCURACY, wh.accuracy_rate(-20)),
             ("fixed_accuracy_2^-14", wh.WH_FMT_ZFP_FIXED_ACCURACY, wh.accuracy_rate(-14))]
    for name, fmt, rate in cases:
        t0 = time.perf_counter()
        if fmt == wh.WH_FMT_ZFP_FIXED_RATE:
            buf = torch.empty(wh.stream_bytes(rows, cols, rate), dtype=torch.uint8, device="cuda")
            wh.wh_encode(ctx, Md, rate, buf)
            torch.cuda.synchronize()
        else:
            buf = torch.from_numpy(wh.wh_encode_var(M, fmt, rate)).cuda()
        t_enc = time.perf_counter() - t0
        m = wh.wh_load_compressed(ctx, rows, cols, fmt, rate, buf)
        t_dec = time_call(lambda i: wh.wh_decode(ctx, m, out), max(3, steps // 4), 1)
        err = (out - Md).double()
        rmse = float(torch.sqrt((err * err).mean()))
        nrmse = rmse / rng
        t_gemv = time_call(lambda i: wh.wh_gemv(ctx, m, u, y, 0, rows), max(5, steps // 2), 2)
        if fmt == wh.WH_FMT_ZFP_FIXED_RATE:
            mhat = sample.decoded(rate)
        elif fmt == wh.WH_FMT_ZFP_FIXED_PRECISION:
            mhat = sample.decoded_var(oracle.VAR_PRECISION, rate)
        else:
            mhat = sample.decoded_var(oracle.VAR_ACCURACY, rate - 1024)
        gerr = err_entry(sample.take(y), mhat @ u64, 1e-6)
        bpv = 8.0 * buf.numel() / (rows * cols)
        res[name] = {"bits_per_value": round(bpv, 3), "ratio": round(32.0 / bpv, 2),
                     "rmse": float(f"{rmse:.4g}"), "nrmse": float(f"{nrmse:.4g}"),
                     "max_error": float(f"{float(err.abs().max()):.4g}"),
                     "psnr": round(-20.0 * math.log10(2.0 * nrmse), 2) if nrmse > 0 else None,
                     "encode_s": round(t_enc, 3), "encoder": "GPU" if fmt == wh.WH_FMT_ZFP_FIXED_RATE else "host",
                     "decode_ms": round(t_dec, 3), "decode_wc_gbs": round(4.0 * rows * cols / (t_dec * 1e-3) / 1e9, 1),
                     "gemv_ms": round(t_gemv, 3), "gemv_error_vs_oracle": gerr,
                     "gemv_effective_gbs": round(4.0 * rows * cols / (t_gemv * 1e-3) / 1e9, 1)}
        wh.wh_unload(ctx, m)
        del buf
    del Md, out
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(size, rate, y_gpu=None):
    """The CPU oracle, as it stands, timed on this host's cores (a baseline,
    not a target), following the plan: decode + FP64 GEMV and decode alone,
    on one core and on all the process's cores (up to 16), for the 4096^2
    matrix at rate 16 (whole matrix, median of 10 runs) and for row samples
    of the 65536^2 matrix at rates 8 and 16 (median of 3).  The oracle's
    GEMV threads over block rows itself; its decode is single-threaded, so
    the all-core decode runs it on equal row chunks from a thread pool.
    Inputs (generation, encoding) are prepared before the clock starts.  With
    y_gpu (the GPU's y for u = the spec's dose vector), also the relative L2
    error of its first rows against the oracle's FP64 GEMV of those rows."""
    import statistics
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    from paper_1902_08018_amd import synth
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    pool = ThreadPoolExecutor(max_workers=cores)

    def chunks(n, parts):
        step = max(4, (n // parts + 3) // 4 * 4)
        return [(r, min(n, r + step)) for r in range(0, n, step)]

    def encode_par(spec, r0, r1, rt):
        table = synth.kernel_table(spec)
        parts = pool.map(lambda c: oracle.encode(synth.matrix_rows(spec, r0 + c[0], r0 + c[1], table), rt),
                         chunks(r1 - r0, cores))
        return np.concatenate(list(parts))

    def median_s(fn, reps):
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
        return statistics.median(t)

    def time_case(spec, code, n, rt, threads, reps, u):
        per = oracle.stream_nbytes(4, spec.cols, rt)
        if threads == 1:
            t_g = median_s(lambda: oracle.gemv_fp64(code, n, spec.cols, rt, u, nthreads=1), reps)
            t_d = median_s(lambda: oracle.decode(code, n, spec.cols, rt), reps)
        else:
            cs = chunks(n, threads)
            t_g = median_s(lambda: oracle.gemv_fp64(code, n, spec.cols, rt, u, nthreads=threads), reps)
            t_d = median_s(lambda: list(pool.map(
                lambda c: oracle.decode(code[c[0] // 4 * per:(c[1] + 3) // 4 * per], c[1] - c[0], spec.cols, rt),
                cs)), reps)
        vals = n * spec.cols
        return {"decode_gemv": {"s": round(t_g, 5), "gflops": round(n * (2 * spec.cols - 1) / t_g / 1e9, 4),
                                "values_per_s": float(f"{vals / t_g:.4g}"),
                                "effective_gbs": round(4.0 * vals / t_g / 1e9, 4)},
                "decode_only": {"s": round(t_d, 5), "values_per_s": float(f"{vals / t_d:.4g}"),
                                "effective_gbs": round(4.0 * vals / t_d / 1e9, 4)}}

    t_all0 = time.perf_counter()
    plan = {}
    # 4096^2, rate 16: the whole matrix, median of 10
    sm = synth.SMALL
    code = encode_par(sm, 0, sm.rows, 16)
    u = synth.u_vector(sm)
    plan["4096x4096_rate16_whole_matrix"] = {
        "all_cores": time_case(sm, code, sm.rows, 16, cores, 10, u),
        "one_core": time_case(sm, code, sm.rows, 16, 1, 10, u), "runs": 10}
    # 65536^2, rates 8 and 16: row samples (whole rows), median of 3
    lg = synth.LARGE
    u = synth.u_vector(lg)
    n_all, n_one = 1024, 64
    for rt in (8, 16):
        code = encode_par(lg, 0, n_all, rt)
        plan[f"65536x65536_rate{rt}_rows_0_{n_all}"] = {
            "all_cores": time_case(lg, code, n_all, rt, cores, 3, u),
            "one_core": dict(time_case(lg, code, n_one, rt, 1, 3, u), rows=f"0..{n_one}"), "runs": 3}
    head = plan[f"65536x65536_rate{rate}_rows_0_{n_all}"]["all_cores"]["decode_gemv"] if size == 65536 else None
    wall = time.perf_counter() - t_all0
    base = {"value": head["effective_gbs"] if head else None,
            "unit": "GB/s effective (uncompressed FP32 bytes/s)", "cores": cores, "kind": "oracle",
            "sample": f"rows 0..{n_all} of the 65536x65536 matrix (all columns), rate {rate}, oracle decode + FP64 "
                      f"GEMV on {cores} threads, median of 3",
            "gflops": head["gflops"] if head else None,
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "threads_used": cores,
            "clock": "wall (perf_counter); generation and encoding excluded",
            "plan": plan, "total_wall_s": round(wall, 1),
            "paper_context": "CPU-MP (AVX2 + OpenMP, uncompressed, Xeon E5-2660 v4): 23.14 GFLOP/s"}
    parity = None
    if y_gpu is not None:
        spec = lg if size == 65536 else synth.MatrixSpec(size, size, int(round(size ** 0.5)), 32.0)
        n = min(len(y_gpu), 256)
        sref = oracle.encode(synth.matrix_rows(spec, 0, n), rate)
        y_ref = oracle.gemv_fp64(sref, n, spec.cols, rate, synth.u_vector(spec), nthreads=cores)
        d = np.asarray(y_gpu[:n], np.float64) - y_ref
        parity = {"rows": f"0..{n}", "rel_l2": float(np.linalg.norm(d) / np.linalg.norm(y_ref)),
                  "max_abs": float(np.abs(d).max()), "tolerance": 1e-6}
    pool.shutdown()
    return base, parity


SERVING_SPECS = {
    "16384x16384": (16384, 16384, 128, 32.0),
    "32768x16384": (32768, 16384, 128, 32.0),
    "65536x65536": (65536, 65536, 256, 32.0),
}


def bench_serving(names=("16384x16384", "32768x16384", "65536x65536"), n_measured=20000, warmup_s=1.0,
                  rate_hz=2000.0, deadline_ms=5.0, budget_mb=512, seed=0, shed=0):
    """Open-loop Poisson load against resident rate-8 matrices (target
    uniform over `names`); k ~ U{1..8} dose vectors in pinned host memory;
    latency measured from the scheduled arrival time."""
    import numpy as np
    import torch
    from paper_1902_08018_amd import synth, wh, workload
    specs = [synth.MatrixSpec(*SERVING_SPECS[n]) for n in names]
    nm = len(specs)
    old = os.environ.pop("WH_SERVE_SHED", None)
    if shed:
        os.environ["WH_SERVE_SHED"] = str(shed)  # read by wh_create
    try:
        ctx = wh.wh_create(0, budget_mb << 20)
    finally:
        os.environ.pop("WH_SERVE_SHED", None)
        if old is not None:
            os.environ["WH_SERVE_SHED"] = old
    streams, mats = [], []
    for sp in specs:
        st = workload.build_stream(ctx, sp, 8)
        streams.append(st)
        mats.append(wh.wh_load_compressed(ctx, sp.rows, sp.cols, wh.WH_FMT_ZFP_FIXED_RATE, 8, st))
    # trace (stream 3): exponential gaps, target matrix, k
    n_warm = int(warmup_s * rate_hz)
    n = n_warm + n_measured
    uu = synth.uniform(3 * n, seed=seed, stream=synth.STREAM_TRACE).astype(np.float64)
    gaps = -np.log1p(-uu[0::3]) / rate_hz
    target = np.minimum((uu[1::3] * nm).astype(int), nm - 1)
    ks = 1 + np.minimum((uu[2::3] * 8).astype(int), 7)
    arrive = np.cumsum(gaps)
    # pinned host buffers, a pool per matrix reused round-robin
    pool = 256
    Ubuf = [torch.from_numpy(synth.uniform(8 * sp.cols, seed=seed + 1).reshape(8, sp.cols)).pin_memory() for sp in specs]
    Ybuf = [[torch.empty((8, sp.rows), dtype=torch.float32).pin_memory() for _ in range(pool)] for sp in specs]
    slot = [0] * nm
    outstanding = {}
    last_done = [None] * nm
    lat, miss, bsz, rejected = [], 0, [], 0
    per = [{"lat": [], "miss": 0, "rejected": 0, "queue": [], "service": []} for _ in range(nm)]
    # the client must not pause: a garbage collection of the lists below
    # took 25-60 ms once per run, during which no request was submitted and
    # every one due meanwhile was late (latency counts from the scheduled
    # arrival)
    import gc
    gc_was_on = gc.isenabled()
    gc.disable()
    t0 = time.monotonic_ns() + 50_000_000
    i = 0
    done_count = 0
    while i < n or outstanding:
        now = time.monotonic_ns()
        while i < n and t0 + int(arrive[i] * 1e9) <= now:
            j = int(target[i])
            k = int(ks[i])
            yslot = slot[j] % pool
            Y = Ybuf[j][yslot]
            slot[j] += 1
            req = wh.wh_request(mat=mats[j], U=Ubuf[j].data_ptr(), u_on_device=0, k=k, Y=Y.data_ptr(), y_on_device=0,
                                deadline_ns=int(deadline_ms * 1e6), arrival_ns=t0 + int(arrive[i] * 1e9))
            try:
                outstanding[wh.wh_submit(ctx, req)] = (i, yslot)
            except wh.WhError:
                rejected += 1
                if i >= n_warm:
                    per[j]["rejected"] += 1
            i += 1
        for tk in list(outstanding):
            st, r = wh.wh_poll(ctx, tk)
            if st == wh.WH_OK:
                idx, yslot = outstanding.pop(tk)
                done_count += 1
                last_done[int(target[idx])] = (idx, yslot)
                if idx >= n_warm:
                    lat.append((r.t_done_ns - r.t_arrive_ns) * 1e-6)
                    miss += r.missed
                    bsz.append(r.batch_size)
                    pj = per[int(target[idx])]
                    pj["lat"].append(lat[-1])
                    pj["miss"] += r.missed
                    pj["queue"].append((r.t_start_ns - r.t_arrive_ns) * 1e-6)   # waiting to join a launch
                    pj["service"].append((r.t_done_ns - r.t_start_ns) * 1e-6)  # one pass of the scan
        if i < n:
            nxt = t0 + int(arrive[i] * 1e9) - time.monotonic_ns()
            if nxt > 200_000:
                time.sleep(min(nxt, 1_000_000) * 1e-9 * 0.5)
    t_total = (time.monotonic_ns() - t0) * 1e-9
    if gc_was_on:
        gc.enable()
    wh.wh_destroy(ctx)
    # the last request each matrix completed, against the oracle on sampled
    # rows (its Y buffer is not reused after it: nothing else is in flight)
    checks = {}
    for j, sp in enumerate(specs):
        if last_done[j] is None:
            continue
        idx, yslot = last_done[j]
        k = int(ks[idx])
        smp = SampledRows(sp, nsample=6)
        ref = Ubuf[j][:k].numpy().astype(np.float64) @ smp.decoded(8).T
        checks[f"{sp.rows}x{sp.cols}"] = dict(err_entry(smp.take(Ybuf[j][yslot][:k].numpy()), ref, 1e-6),
                                              request=int(idx), k=k)
    lat = np.array(lat)
    return {"requests": int(len(lat)), "rate_hz": rate_hz, "deadline_ms": deadline_ms,
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "p999_ms": round(float(np.percentile(lat, 99.9)), 3), "max_ms": round(float(lat.max()), 3),
            "miss_rate": round(miss / max(1, len(lat)), 4), "throughput_rps": round(done_count / t_total, 1),
            "mean_batch_requests": round(float(np.mean(bsz)), 2), "rejected": rejected,
            "hbm_budget_mb": budget_mb, "shed_after_deadlines": shed,
            "matrices": [f"{sp.rows}x{sp.cols} rate 8" for sp in specs],
            "last_result_error_vs_oracle": checks,
            "per_matrix": {f"{sp.rows}x{sp.cols}": {"requests": len(pj["lat"]),
                                                   "p50_ms": round(float(np.percentile(pj["lat"], 50)), 3),
                                                   "p99_ms": round(float(np.percentile(pj["lat"], 99)), 3),
                                                   "miss_rate": round(pj["miss"] / max(1, len(pj["lat"])), 4),
                                                   "rejected": pj["rejected"],
                                                   "queue_p50_ms": round(float(np.percentile(pj["queue"], 50)), 3),
                                                   "service_p50_ms": round(float(np.percentile(pj["service"], 50)),
                                                                          3),
                                                   "service_p99_ms": round(float(np.percentile(pj["service"], 99)),
                                                                          3)}
                           for sp, pj in zip(specs, per) if pj["lat"]}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (--gpus {args.gpus} requested); "
              "the row split across GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1902_08018_amd import synth, wh, workload

    size, rate = args.size, args.rate
    spec = synth.LARGE if size == 65536 else synth.MatrixSpec(size, size, int(round(size ** 0.5)), 32.0)
    rows, cols = spec.rows, spec.cols
    if args.leg == "serving":
        print(json.dumps(bench_serving(n_measured=args.serving_requests)), flush=True)
        return
    ctx = wh.wh_create(0, 0)
    if args.leg == "thermal":
        print(json.dumps(bench_thermal(ctx, args.steps)), flush=True)
        wh.wh_destroy(ctx)
        return
    if args.leg == "var":
        global VAR_SPEC_ARGS
        VAR_SPEC_ARGS = (args.var_size, args.var_size) + tuple(VAR_SPEC_ARGS[2:])
        print(json.dumps(bench_var(ctx, args.steps)), flush=True)
        wh.wh_destroy(ctx)
        return
    if args.leg == "host-pipeline":
        print(json.dumps(bench_host_pipeline(ctx, rate, args.steps)), flush=True)
        wh.wh_destroy(ctx)
        return
    print(f"# building rate-{rate} stream of {rows}x{cols} on the GPU", file=sys.stderr, flush=True)
    stream = workload.build_stream(ctx, spec, rate)
    mat = wh.wh_load_compressed(ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, rate, stream)
    us = [workload.u_device(spec, synth.STREAM_U, k * cols) for k in range(4)]
    y = torch.empty(rows, dtype=torch.float32, device="cuda")
    if args.probe == 2:
        k = args.probe_k
        U = torch.from_numpy(synth.u_batch(spec, k)).cuda()
        if args.probe_bf16:
            U = U.to(torch.bfloat16)
        Y = torch.empty((k, rows), dtype=torch.float32, device="cuda")
        for _ in range(3):
            wh.wh_gemv_batched(ctx, mat, U, Y)
        torch.cuda.synchronize()
        print(f"# probe done: 3 x wh_gemv_batched k={k} {'BF16' if args.probe_bf16 else 'FP32'} U rate {rate} "
              f"{rows}x{cols}", file=sys.stderr, flush=True)
        wh.wh_destroy(ctx)
        return
    if args.probe == 3:
        dense = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
        for _ in range(3):
            wh.wh_decode(ctx, mat, dense)
        torch.cuda.synchronize()
        print(f"# probe done: 3 x wh_decode rate {rate} {rows}x{cols}", file=sys.stderr, flush=True)
        wh.wh_destroy(ctx)
        return
    if args.probe:
        for i in range(3):
            wh.wh_gemv(ctx, mat, us[i], y, 0, rows, args.flags)
        torch.cuda.synchronize()
        a = torch.ones(1 << 30, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        xo = torch.zeros(1, dtype=torch.int32, device="cuda")
        for _ in range(3):
            wh.wh_stream_read(ctx, a, xo)
        torch.cuda.synchronize()
        print(f"# probe done: 3 x wh_gemv rate {rate} {rows}x{cols}, 3 x copy and 3 x read-only stream of "
              f"{a.numel() * 4} bytes",
              file=sys.stderr, flush=True)
        wh.wh_destroy(ctx)
        return
    print("# timing", file=sys.stderr, flush=True)
    wall_ms, ev_ms = time_gemv(ctx, mat, us, y, rows, args.steps, args.warmup, args.flags)
    kern_ms = sum(ev_ms) / len(ev_ms)
    stream_bytes = stream.numel()
    alg_bytes = stream_bytes + 4 * cols + 4 * rows
    eff_gbs = 4.0 * rows * cols / (wall_ms * 1e-3) / 1e9
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    flop = rows * (2 * cols - 1)
    # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter passes,
    # valid only for the kernel source they were taken on
    traffic = valu_insts = None
    try:
        with open(args.traffic_json) as f:
            tj = json.load(f).get(f"whz_gemv_rate{rate}_{rows}x{cols}")
        if tj and tj.get("kernel_source_sha256_16") == kernel_source_hash():
            traffic = tj.get("bytes_per_launch")
            valu_insts = tj.get("sq_insts_valu")
    except (OSError, ValueError):
        pass
    # the timed configuration once more with u = the spec's dose vector: its
    # first rows go to the oracle's check
    wh.wh_gemv(ctx, mat, us[0], y, 0, rows, args.flags)
    torch.cuda.synchronize()
    y_head = y[:PARITY_ROWS].cpu().numpy()
    # the box's streaming ceiling: a plain 4 GiB device-to-device copy
    ca = torch.empty(1 << 30, dtype=torch.int32, device="cuda").fill_(1)
    cb = torch.empty_like(ca)
    copy_ms = time_call(lambda i: cb.copy_(ca), 5, 2)
    copy_gbs = 2 * ca.numel() * 4 / (copy_ms * 1e-3) / 1e9
    # and the read-only ceiling: the library's streaming probe reads 4 GiB once
    xo = torch.zeros(1, dtype=torch.int32, device="cuda")
    read_ms = time_call(lambda i: wh.wh_stream_read(ctx, ca, xo), 5, 2)
    read_gbs = ca.numel() * 4 / (read_ms * 1e-3) / 1e9
    del ca, cb
    out = {
        "metric": "decode+GEMV effective GB/s (frac of HBM peak), GFLOP/s; p99 latency vs deadline",
        "value": round(eff_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fused WHZ1 decode+GEMV, {rows}x{cols} FP32 response matrix "
                               f"(256x256 lattices, ell 32, sigma 1e-4), zfp-style fixed rate {rate} bits/value "
                               f"({stream_bytes / 1e9:.2f} GB resident), u 65536 U[0,1)",
                   "rate": rate, "rows": rows, "cols": cols, "acc": "fp64" if args.flags in (0, 1) else args.flags,
                   "parallelism": "single GPU"},
        "gflops": round(flop / (wall_ms * 1e-3) / 1e9, 2),
        "compressed_gbs": round(stream_bytes / (kern_ms * 1e-3) / 1e9, 2),
        "kernel_ms": round(kern_ms, 4),
        "kernel_ms_p10_p50_p90": [round(float(x), 4) for x in __import__("numpy").percentile(ev_ms, [10, 50, 90])],
        "paper_context": {"p100_zfp_decoder_wc_gbs": 33.2, "p100_mixed_precision_gemv_gflops": 198.3,
                          "note": "the paper's own P100 figures (separate zfp decoder, fixed accuracy; uncompressed "
                                  "378 x 256000 GEMV): context, not this metric's baseline"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "copy_ceiling_gbs": round(copy_gbs, 1), "read_ceiling_gbs": round(read_gbs, 1),
                     "frac_of_read_ceiling": round(achieved / read_gbs, 4)},
    }
    if valu_insts:
        # the decoder's VALU work: 64 lanes per wave64 instruction
        # (SQ_INSTS_VALU of a counter run on this kernel source) over this run's
        # kernel time, against the chip's vector rate
        ops = valu_insts * 64
        out["roofline"]["valu"] = {"lane_ops_per_launch": ops, "achieved": round(ops / (kern_ms * 1e-3) / 1e12, 2),
                                   "peak": VALU_PEAK_TOPS, "unit": "T lane-ops/s",
                                   "frac": round(ops / (kern_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4)}
    wh.wh_unload(ctx, mat)
    del stream
    torch.cuda.empty_cache()

    if args.extra:
        import numpy as np
        extra = {}
        print("# oracle references for sampled rows", file=sys.stderr, flush=True)
        sample = SampledRows(spec)
        u64 = synth.u_vector(spec).astype(np.float64)
        extra["sampled_rows_for_errors"] = (f"{len(sample.idx)} rows in {len(sample.brows)} block rows spread over "
                                            f"0..{rows}; references: the oracle's FP64 products")
        # rate 16 on the same matrix
        print("# rate 16", file=sys.stderr, flush=True)
        s16 = workload.build_stream(ctx, spec, 16)
        m16 = wh.wh_load_compressed(ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, 16, s16)
        w16, e16 = time_gemv(ctx, m16, us, y, rows, max(5, args.steps // 2), 2, args.flags)
        k16 = sum(e16) / len(e16)
        wh.wh_gemv(ctx, m16, us[0], y, 0, rows, args.flags)
        extra["rate16"] = {"effective_gbs": round(4.0 * rows * cols / (k16 * 1e-3) / 1e9, 2),
                           "kernel_ms": round(k16, 4),
                           "hbm_frac": round((s16.numel() + 8 * cols) / (k16 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "gflops": round(flop / (k16 * 1e-3) / 1e9, 2),
                           "error_vs_oracle": err_entry(sample.take(y), sample.decoded(16) @ u64, 1e-6)}
        # separate path: decode to dense FP32, then dense GEMV (rate 8)
        print("# separate path", file=sys.stderr, flush=True)
        wh.wh_unload(ctx, m16)
        del s16
        torch.cuda.empty_cache()
        s8 = workload.build_stream(ctx, spec, rate)
        m8 = wh.wh_load_compressed(ctx, rows, cols, wh.WH_FMT_ZFP_FIXED_RATE, rate, s8)
        dense = torch.empty((rows, cols), dtype=torch.float32, device="cuda")
        dm = wh.wh_load_compressed(ctx, rows, cols, wh.WH_FMT_F32, 0, dense)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        for _ in range(2):
            wh.wh_decode(ctx, m8, dense)
            wh.wh_gemv(ctx, dm, us[0], y, 0, rows)
        torch.cuda.synchronize()
        reps = 3
        td = tg = 0.0
        for i in range(reps):
            e0.record()
            wh.wh_decode(ctx, m8, dense)
            e1.record()
            wh.wh_gemv(ctx, dm, us[i % 4], y, 0, rows)
            e2.record()
            torch.cuda.synchronize()
            td += e0.elapsed_time(e1)
            tg += e1.elapsed_time(e2)
        td, tg = td / reps, tg / reps
        wh.wh_gemv(ctx, dm, us[0], y, 0, rows)
        dec_rows = dense[torch.from_numpy(sample.idx).cuda()].cpu().numpy()
        extra["separate_rate8"] = {"decode_ms": round(td, 4), "dense_gemv_ms": round(tg, 4),
                                   "total_ms": round(td + tg, 4),
                                   "effective_gbs": round(4.0 * rows * cols / ((td + tg) * 1e-3) / 1e9, 2),
                                   "dense_gemv_hbm_frac": round((4.0 * rows * cols + 8 * cols) / (tg * 1e-3) / 1e9
                                                                / HBM_PEAK_GBS, 4),
                                   "decode_bitexact_on_sampled_rows": bool(np.array_equal(
                                       dec_rows.view(np.uint32),
                                       sample.decoded(rate).astype(np.float32).view(np.uint32))),
                                   "error_vs_oracle": err_entry(sample.take(y), sample.decoded(rate) @ u64, 1e-6)}
        # one GPU's share of an 8-way row split (the sharded layout needs no
        # exchange: each GPU owns 8192 rows of the stream and of y)
        print("# row shard", file=sys.stderr, flush=True)
        shard = {}
        for r0 in (0, rows - rows // 8):
            ms = time_call(lambda i: wh.wh_gemv(ctx, m8, us[i % 4], y[: rows // 8], r0, r0 + rows // 8),
                           max(5, args.steps // 2), 2)
            wh.wh_gemv(ctx, m8, us[0], y[: rows // 8], r0, r0 + rows // 8)
            sel = (sample.idx >= r0) & (sample.idx < r0 + rows // 8)
            got = y[torch.from_numpy(sample.idx[sel] - r0).cuda()].cpu().numpy()
            shard[f"rows_{r0}_{r0 + rows // 8}"] = {"ms": round(ms, 4),
                                                   "effective_gbs": round(4.0 * rows // 8 * cols / (ms * 1e-3) / 1e9, 1),
                                                   "error_vs_oracle": err_entry(got, (sample.decoded(rate) @ u64)[sel],
                                                                                1e-6)}
        extra["row_shard_1_of_8_rate8"] = shard
        print("# multi-RHS", file=sys.stderr, flush=True)
        extra["multi_rhs_rate8"] = bench_multi_rhs(ctx, m8, spec, rate, s8.numel(), max(3, args.steps // 4), sample)
        out["extra"] = extra
        wh.wh_unload(ctx, dm)
        wh.wh_unload(ctx, m8)
        del dense, s8
        torch.cuda.empty_cache()
        print("# dense precision sweep", file=sys.stderr, flush=True)
        extra["dense_precision"] = bench_precision(ctx, spec, us, y, max(5, args.steps // 2), sample)
        print("# the paper's GEMV shapes and slit windows of a field matrix", file=sys.stderr, flush=True)
        extra[f"slit_field_rate{rate}"] = bench_slit_field(ctx, rate, max(10, args.steps))
        print("# host-resident matrices streamed over the link (child process)", file=sys.stderr, flush=True)
        hp = host_pipeline_child(rate, max(5, args.steps // 2))
        print("# the same pipeline in this process, after the other legs", file=sys.stderr, flush=True)
        hctx = wh.wh_create(0, 0)  # its copy stream (a hardware queue) goes with it
        hp["in_process_after_other_legs"] = bench_host_pipeline(hctx, rate, max(5, args.steps // 2),
                                                                modes=("chunk_32MiB",), parts=False)
        wh.wh_destroy(hctx)
        extra[f"host_pipeline_rate{rate}"] = hp
        print("# thermal step", file=sys.stderr, flush=True)
        extra["thermal_step_608x608"] = bench_thermal(ctx, args.steps)
        print("# variable-rate modes", file=sys.stderr, flush=True)
        extra["variable_rate_8192x8192"] = bench_var(ctx, args.steps)

    if args.serving:
        print("# serving loop", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out.setdefault("extra", {})["serving"] = bench_serving(n_measured=args.serving_requests)
        # the same arrival process on the two smaller matrices only: one pass
        # over the 65536^2 matrix takes longer than the deadline by itself
        print("# serving loop, two smaller matrices", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["extra"]["serving_two_smaller"] = bench_serving(("16384x16384", "32768x16384"),
                                                            n_measured=args.serving_requests)
        # the three matrices again, shedding requests for a matrix whose queue
        # head has waited more than four deadlines
        print("# serving loop, load shedding", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["extra"]["serving_shed_4"] = bench_serving(n_measured=args.serving_requests, shed=4)

    if args.cpu_baseline:
        print("# cpu baseline (oracle), and the oracle's check of the timed launch's first rows",
              file=sys.stderr, flush=True)
        out["cpu_baseline"], out["parity_vs_oracle"] = cpu_baseline(size, rate, y_head)
    wh.wh_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
