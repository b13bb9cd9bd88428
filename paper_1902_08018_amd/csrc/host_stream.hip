// host_stream.hip -- fused decode + GEMV over a compressed matrix that stays
// in host memory.
//
// The paper keeps the whole model matrix in host DDR and moves it to the GPU
// over PCIe compressed, with the transfers pipelined against the work on the
// GPU (Sec. 4.2 and 4.3, Table 1: with compression the period is
// max(T_transfer / R, T_compute + T_decode)).  Here the block rows of the
// requested range cross the link in chunks on a copy stream of the library's,
// into two device staging buffers used in turn; the fused decode + GEMV of a
// chunk runs on the caller's stream as soon as its copy has landed, while the
// next chunk is in flight.  The decode and the GEMV are one kernel, so
// T_compute + T_decode is the fused kernel's time on the chunk.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/wh.h"
#include "wh_ctx.hpp"
#include "wh_internal.hpp"

namespace wh {

struct HostPipe {
    hipStream_t copy = nullptr;
    void* buf[kPipeBuffers] = {};
    size_t buf_bytes = 0;
    hipEvent_t copied[kPipeBuffers] = {};
    hipEvent_t consumed[kPipeBuffers] = {};
    hipEvent_t entry = nullptr;
};

void host_pipe_free(wh_ctx* ctx)
{
    HostPipe* p = ctx->pipe;
    if (!p)
        return;
    if (p->copy)
        (void)hipStreamSynchronize(p->copy);
    for (int k = 0; k < kPipeBuffers; ++k) {
        if (p->buf[k])
            (void)hipFree(p->buf[k]);
        if (p->copied[k])
            (void)hipEventDestroy(p->copied[k]);
        if (p->consumed[k])
            (void)hipEventDestroy(p->consumed[k]);
    }
    if (p->entry)
        (void)hipEventDestroy(p->entry);
    if (p->copy)
        (void)hipStreamDestroy(p->copy);
    delete p;
    ctx->pipe = nullptr;
}

namespace {

// The copy stream, events and staging buffers of at least `bytes` each.
wh_status ensure_pipe(wh_ctx* ctx, size_t bytes)
{
    if (!ctx->pipe) {
        HostPipe* p = new HostPipe();
        ctx->pipe = p;
        hipError_t e = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking);
        for (int k = 0; k < kPipeBuffers && e == hipSuccess; ++k) {
            e = hipEventCreateWithFlags(&p->copied[k], hipEventDisableTiming);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&p->consumed[k], hipEventDisableTiming);
        }
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&p->entry, hipEventDisableTiming);
        if (e != hipSuccess) {
            host_pipe_free(ctx);
            return device_error(ctx, e);
        }
    }
    HostPipe* p = ctx->pipe;
    if (bytes <= p->buf_bytes)
        return WH_OK;
    // the old buffers may still be read by queued work
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return device_error(ctx, e);
    for (int k = 0; k < kPipeBuffers; ++k) {
        if (p->buf[k])
            (void)hipFree(p->buf[k]);
        p->buf[k] = nullptr;
    }
    p->buf_bytes = 0;
    for (int k = 0; k < kPipeBuffers; ++k) {
        e = hipMalloc(&p->buf[k], bytes);
        if (e != hipSuccess) {
            for (int j = 0; j < kPipeBuffers; ++j) {
                if (p->buf[j])
                    (void)hipFree(p->buf[j]);
                p->buf[j] = nullptr;
            }
            return device_error(ctx, e);
        }
    }
    p->buf_bytes = bytes;
    return WH_OK;
}

} // namespace


namespace {

// Chunk c covers block rows [bb + c * cb, min(bb + (c + 1) * cb, be)) of the
// matrix; as a matrix of its own it has rows [4 * b0, min(4 * b1, rows)).
struct Chunk {
    uint32_t r0;   // first matrix row of the chunk
    uint32_t rows; // its rows
    uint32_t lo;   // the requested range inside the chunk: [lo, hi)
    uint32_t hi;
};

Chunk chunk_at(uint32_t b0, uint32_t b1, uint32_t rows, uint32_t row_begin, uint32_t row_end)
{
    Chunk c;
    c.r0 = 4 * b0;
    c.rows = std::min(4 * b1, rows) - c.r0;
    c.lo = std::max(row_begin, c.r0) - c.r0;
    c.hi = std::min(row_end, c.r0 + c.rows) - c.r0;
    return c;
}

} // namespace

} // namespace wh

using namespace wh;

extern "C" wh_status wh_gemv_host(wh_ctx* ctx, const void* h_code, uint32_t rows, uint32_t cols, uint32_t rate,
                                  const float* d_u, float* d_y, uint32_t row_begin, uint32_t row_end,
                                  uint32_t chunk_rows, uint32_t flags, void* stream)
{
    WH_GUARD(ctx);
    if (!h_code || !d_u || !d_y || !aligned(d_u, 16) || chunk_rows % 4)
        return WH_ERR_INVALID;
    if (flags & ~(WH_ACC_FP64 | WH_ACC_TWOSUM | WH_PAPER_MP | WH_HOST_DIRECT))
        return WH_ERR_INVALID;
    if ((flags & WH_ACC_FP64) && (flags & WH_ACC_TWOSUM))
        return WH_ERR_INVALID;
    if (rows == 0 || cols == 0)
        return WH_ERR_SHAPE;
    if (!whz_rate_supported(rate))
        return WH_ERR_FORMAT;
    if (row_begin > row_end || row_end > rows)
        return WH_ERR_SHAPE;
    if (row_begin == row_end)
        return WH_OK;
    try {
        const AccMode mode = (flags & WH_PAPER_MP)     ? AccMode::PaperMp
                             : (flags & WH_ACC_TWOSUM) ? AccMode::TwoSum
                                                       : AccMode::Fp64;
        const uint64_t brow_bytes = (uint64_t)((cols + 3) / 4) * 2u * rate; // one block row of code
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (flags & WH_HOST_DIRECT) {
            // the fused kernel reads the page-locked stream over the link
            // itself: no staging, no copy engine
            void* dev = nullptr;
            if (hipHostGetDevicePointer(&dev, const_cast<void*>(h_code), 0) != hipSuccess || !dev) {
                (void)hipGetLastError();
                return WH_ERR_INVALID;
            }
            const GemvPlan pl = whz_gemv_plan(rate, rows, cols, row_begin, row_end, ctx->num_cus, &ctx->gemv_tune);
            if (pl.nslab > 1) {
                const wh_status s = ensure_partials(ctx, (size_t)pl.nslab * pl.part_rows(), st);
                if (s != WH_OK)
                    return s;
            }
            const hipError_t e = whz_gemv(rate, pl, mode, dev, d_u, d_y, pl.nslab > 1 ? ctx->part : nullptr, st);
            return device_error(ctx, pl.nslab > 1 ? partials_release(ctx, st, e) : e);
        }
        const uint32_t bb = row_begin / 4, be = (row_end + 3) / 4;
        uint64_t cb = chunk_rows ? chunk_rows / 4 : kPipeChunkBytes / brow_bytes;
        cb = std::max<uint64_t>(1, std::min<uint64_t>(cb, be - bb));
        wh_status s = ensure_pipe(ctx, (size_t)(cb * brow_bytes));
        if (s != WH_OK)
            return s;
        // FP64 slab partials: every chunk's plan shares the context's
        // workspace, in stream order
        // (the first and last chunks plan on their own, the others alike)
        size_t part_need = 0;
        const uint64_t nchunks = (be - bb + cb - 1) / cb;
        for (uint64_t n : {(uint64_t)0, (uint64_t)1, nchunks - 1}) {
            if (n >= nchunks)
                continue;
            const uint64_t b0 = bb + n * cb;
            const uint32_t b1 = (uint32_t)std::min<uint64_t>(b0 + cb, be);
            const Chunk c = chunk_at((uint32_t)b0, b1, rows, row_begin, row_end);
            const GemvPlan pl = whz_gemv_plan(rate, c.rows, cols, c.lo, c.hi, ctx->num_cus, &ctx->gemv_tune);
            if (pl.nslab > 1)
                part_need = std::max(part_need, (size_t)pl.nslab * pl.part_rows());
        }
        if (part_need) {
            s = ensure_partials(ctx, part_need, st);
            if (s != WH_OK)
                return s;
        }
        HostPipe* p = ctx->pipe;
        const char* src = static_cast<const char*>(h_code);
        // copies start after the work already on the caller's stream, and
        // after the GEMVs of an earlier call (on any stream) that read the
        // staging buffers
        hipError_t e = hipEventRecord(p->entry, st);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(p->copy, p->entry, 0);
        for (int j = 0; j < kPipeBuffers && e == hipSuccess; ++j)
            e = hipStreamWaitEvent(p->copy, p->consumed[j], 0);
        uint32_t k = 0;
        for (uint64_t b0 = bb, n = 0; b0 < be && e == hipSuccess; b0 += cb, ++n, k = (k + 1) % kPipeBuffers) {
            const uint32_t b1 = (uint32_t)std::min<uint64_t>(b0 + cb, be);
            if (n >= (uint64_t)kPipeBuffers) // the GEMV that last read buffer k is done
                e = hipStreamWaitEvent(p->copy, p->consumed[k], 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(p->buf[k], src + b0 * brow_bytes, (size_t)((b1 - b0) * brow_bytes),
                                   hipMemcpyHostToDevice, p->copy);
            if (e == hipSuccess)
                e = hipEventRecord(p->copied[k], p->copy);
            if (e == hipSuccess)
                e = hipStreamWaitEvent(st, p->copied[k], 0);
            if (e != hipSuccess)
                break;
            const Chunk c = chunk_at((uint32_t)b0, b1, rows, row_begin, row_end);
            const GemvPlan pl = whz_gemv_plan(rate, c.rows, cols, c.lo, c.hi, ctx->num_cus, &ctx->gemv_tune);
            e = whz_gemv(rate, pl, mode, p->buf[k], d_u, d_y + (c.r0 + c.lo - row_begin),
                         pl.nslab > 1 ? ctx->part : nullptr, st);
            if (e == hipSuccess)
                e = hipEventRecord(p->consumed[k], st);
        }
        return device_error(ctx, part_need ? partials_release(ctx, st, e) : e);
    } catch (const std::bad_alloc&) {
        return WH_ERR_NOMEM;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

extern "C" wh_status wh_host_alloc(uint64_t bytes, void** h_ptr)
{
    if (!h_ptr || bytes == 0)
        return WH_ERR_INVALID;
    *h_ptr = nullptr;
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, (size_t)bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return WH_ERR_NOMEM;
    }
    *h_ptr = p;
    return WH_OK;
}

extern "C" wh_status wh_host_free(void* h_ptr)
{
    if (!h_ptr)
        return WH_OK;
    return hipHostFree(h_ptr) == hipSuccess ? WH_OK : WH_ERR_INVALID;
}
