// wh_api.hip -- the C ABI of libwh (declared in include/wh.h).
//
// Context = one HIP device, a table of resident matrices, and workspaces
// (FP64 slab partials of the fused GEMV).  Every entry point validates its
// arguments before anything is launched, returns a wh_status, and never lets
// a C++ exception escape.  A failed HIP call marks the context failed
// (sticky): later calls return WH_ERR_DEVICE.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <mutex>
#include <new>
#include <unordered_map>

#include "../../include/wh.h"
#include "wh_internal.hpp"
#include "wh_ctx.hpp"

using namespace wh;

namespace wh {

wh_status device_error(wh_ctx* ctx, hipError_t e)
{
    if (e == hipSuccess)
        return WH_OK;
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return WH_ERR_NOMEM;
    }
    ctx->failed.store(true);
    return WH_ERR_DEVICE;
}

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

// WH_GEMV_LANES / WH_GEMV_ROWS / WH_GEMV_SLABS fix the fused GEMV's lanes per
// block row, block rows per lane group and column slabs, WH_MRHS_SLABS the
// multi-RHS kernel's column slabs (launch-shape sweeps and tests); a value
// that is not valid is ignored.
GemvTuning gemv_tuning_from_env()
{
    auto get = [](const char* name) -> uint32_t {
        const char* v = std::getenv(name);
        if (!v || !*v)
            return 0;
        char* end = nullptr;
        const unsigned long x = std::strtoul(v, &end, 10);
        return (*end == 0 && x <= 0xFFFFFFFFul) ? (uint32_t)x : 0u;
    };
    GemvTuning t;
    const uint32_t lanes = get("WH_GEMV_LANES"), rows = get("WH_GEMV_ROWS");
    if (lanes >= 4 && lanes <= kGemvLanes && (lanes & (lanes - 1)) == 0)
        t.lanes = lanes;
    if (rows == 1 || rows == 2 || rows == 4)
        t.rows = rows;
    t.slabs = get("WH_GEMV_SLABS");
    t.mrhs_slabs = get("WH_MRHS_SLABS");
    t.mrhs_fp32 = get("WH_MRHS_FP32") ? 1u : 0u;
    return t;
}

// WH_SERVE_CHUNK_VALUES: the most matrix values one serving launch covers
// (a served pass runs as row chunks of about this size); default 2^28.
uint64_t serve_chunk_from_env()
{
    const char* v = std::getenv("WH_SERVE_CHUNK_VALUES");
    if (!v || !*v)
        return 1ull << 28;
    char* end = nullptr;
    const unsigned long long x = std::strtoull(v, &end, 10);
    return (*end == 0 && x > 0) ? (uint64_t)x : (1ull << 28);
}

wh_status storage_bytes(const wh_matrix_desc& d, uint64_t& nbytes)
{
    if (d.rows == 0 || d.cols == 0)
        return WH_ERR_SHAPE;
    if (d.fmt == WH_FMT_ZFP_FIXED_RATE) { // partial blocks at the edges are edge-padded
        if (!whz_rate_supported(d.rate))
            return WH_ERR_FORMAT;
        nbytes = (uint64_t)((d.rows + 3) / 4) * ((d.cols + 3) / 4) * 2u * d.rate;
        return WH_OK;
    }
    if (d.rows % 4 || d.cols % 4) // dense formats: whole 4 x 4 tiles
        return d.fmt >= WH_FMT_F32 && d.fmt <= WH_FMT_FP8E4M3_BS4 ? WH_ERR_SHAPE : WH_ERR_FORMAT;
    const uint64_t n = (uint64_t)d.rows * d.cols;
    const uint64_t nb = n / 16;
    switch (d.fmt) {
    case WH_FMT_F32:
        nbytes = n * 4;
        return WH_OK;
    case WH_FMT_F16:
    case WH_FMT_BF16:
        nbytes = n * 2;
        return WH_OK;
    case WH_FMT_FP8E4M3_BS4:
        nbytes = nb * 16 + nb * 4;
        return WH_OK;
    default:
        return WH_ERR_FORMAT;
    }
}

wh_status grow_partials(wh_ctx* ctx, size_t count);

bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

wh_status ensure_partials(wh_ctx* ctx, size_t count, hipStream_t st)
{
    // a later call may grow the workspace, freeing the memory a captured
    // graph would go on using: calls that need it are not captured
    // (wh_gemv_noalloc is the capturable form)
    if (capturing(st))
        return WH_ERR_INVALID;
    if (count > ctx->part_cap) {
        const wh_status s = grow_partials(ctx, count);
        if (s != WH_OK)
            return s;
    }
    return device_error(ctx, hipStreamWaitEvent(st, ctx->part_ev, 0));
}

hipError_t partials_release(wh_ctx* ctx, hipStream_t st, hipError_t e)
{
    if (e != hipSuccess)
        return e;
    return hipEventRecord(ctx->part_ev, st);
}

wh_status grow_partials(wh_ctx* ctx, size_t count)
{
    if (ctx->part) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess)
            return device_error(ctx, e);
        (void)hipFree(ctx->part);
        ctx->part = nullptr;
        ctx->part_cap = 0;
    }
    size_t cap = count < (1u << 16) ? (1u << 16) : count;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ctx->part), cap * sizeof(double));
    if (e != hipSuccess) {
        ctx->part = nullptr;
        return device_error(ctx, e);
    }
    ctx->part_cap = cap;
    return WH_OK;
}

Matrix* find_matrix(wh_ctx* ctx, wh_mat m)
{
    auto it = ctx->mats.find(m);
    return it == ctx->mats.end() ? nullptr : &it->second;
}

} // namespace wh



extern "C" {

const char* wh_status_str(wh_status st)
{
    switch (st) {
    case WH_OK:
        return "ok";
    case WH_PENDING:
        return "pending";
    case WH_ERR_INVALID:
        return "invalid argument";
    case WH_ERR_SHAPE:
        return "bad shape (rows/cols must be positive multiples of 4; row range multiple of 4)";
    case WH_ERR_FORMAT:
        return "unsupported format, rate or byte count";
    case WH_ERR_NOMEM:
        return "device out of memory";
    case WH_ERR_BUDGET:
        return "request exceeds the HBM budget";
    case WH_ERR_DEVICE:
        return "HIP device error (context failed)";
    case WH_ERR_NOT_FOUND:
        return "unknown matrix handle or ticket";
    case WH_ERR_SCRATCH:
        return "the call needs more workspace than wh_gemv_noalloc's fixed scratch array holds";
    default:
        return "unknown status";
    }
}

wh_status wh_create(int hip_device, uint64_t hbm_budget_bytes, wh_ctx** out)
{
    if (!out)
        return WH_ERR_INVALID;
    try {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
            (void)hipGetLastError();
            return WH_ERR_DEVICE;
        }
        if (hip_device < 0 || hip_device >= ndev)
            return WH_ERR_INVALID;
        if (hipSetDevice(hip_device) != hipSuccess)
            return WH_ERR_DEVICE;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess)
            return WH_ERR_DEVICE;
        // the device address of wh_gemv_noalloc's scratch array on this device
        if (noalloc_init(hip_device) != WH_OK)
            return WH_ERR_DEVICE;
        wh_ctx* ctx = new wh_ctx();
        ctx->device = hip_device;
        ctx->num_cus = prop.multiProcessorCount;
        ctx->gemv_tune = gemv_tuning_from_env();
        ctx->serve_chunk_values = serve_chunk_from_env();
        if (const char* v = std::getenv("WH_SERVE_PACE")) {
            char* end = nullptr;
            const double f = std::strtod(v, &end);
            if (*v && *end == 0 && f >= 1.0 && f <= 16.0)
                ctx->serve_pace = f;
        }
        if (const char* v = std::getenv("WH_SERVE_MARGIN_US")) {
            char* end = nullptr;
            const double f = std::strtod(v, &end);
            if (*v && *end == 0 && f >= 0.0 && f <= 1e6)
                ctx->serve_margin_ns = f * 1e3;
        }
        if (const char* v = std::getenv("WH_SERVE_SHED")) {
            char* end = nullptr;
            const unsigned long f = std::strtoul(v, &end, 10);
            ctx->serve_shed = (*v && *end == 0 && f <= 1000) ? (uint32_t)f : 0u;
        }
        ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (1ull << 30);
        if (hipEventCreateWithFlags(&ctx->part_ev, hipEventDisableTiming) != hipSuccess) {
            delete ctx;
            return WH_ERR_DEVICE;
        }
        // the host pipeline's copy stream is created on its first use: a
        // stream holds a hardware queue (HIP maps streams onto a few queues
        // round-robin), and most contexts never stream from the host
        *out = ctx;
        return WH_OK;
    } catch (const std::bad_alloc&) {
        return WH_ERR_NOMEM;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_destroy(wh_ctx* ctx)
{
    if (!ctx)
        return WH_ERR_INVALID;
    try {
        (void)hipSetDevice(ctx->device);
        serve_shutdown(ctx);
        (void)hipDeviceSynchronize();
        host_pipe_free(ctx);
        for (auto& kv : ctx->mats)
            if (kv.second.owned && kv.second.dptr)
                (void)hipFree(kv.second.dptr);
        if (ctx->part)
            (void)hipFree(ctx->part);
        if (ctx->part_ev)
            (void)hipEventDestroy(ctx->part_ev);
        delete ctx;
        return WH_OK;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_gemv_plan_info(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus,
                            uint32_t rate, uint32_t* out9)
{
    if (!out9 || rows == 0 || cols == 0 || row_begin > row_end || row_end > rows || !whz_rate_supported(rate))
        return WH_ERR_INVALID;
    GemvTuning none;
    const GemvPlan pl = whz_gemv_plan(rate, rows, cols, row_begin, row_end, num_cus, &none);
    const uint32_t v[9] = {1u << pl.lg, pl.rpg, pl.ntiles,  pl.nslab, pl.slab_bc,
                           pl.bi_begin, pl.bi_end, pl.skip, pl.lanes};
    for (int i = 0; i < 9; ++i)
        out9[i] = v[i];
    return WH_OK;
}

wh_status wh_storage_bytes(const wh_matrix_desc* desc, uint64_t* nbytes)
{
    if (!desc || !nbytes)
        return WH_ERR_INVALID;
    uint64_t n = 0;
    wh_status st = storage_bytes(*desc, n);
    if (st == WH_OK)
        *nbytes = n;
    return st;
}

wh_status wh_load_compressed(wh_ctx* ctx, const wh_matrix_desc* desc, const void* bytes, uint64_t nbytes, int where,
                             wh_mat* out)
{
    WH_GUARD(ctx);
    if (!desc || !bytes || !out || (where != WH_HOST && where != WH_DEVICE))
        return WH_ERR_INVALID;
    try {
        uint64_t need = 0;
        int vmode = 0, vparam = 0;
        if (desc->fmt == WH_FMT_ZFP_FIXED_PRECISION || desc->fmt == WH_FMT_ZFP_FIXED_ACCURACY) {
            // variable length: the index, then at least the reader's padding
            if (desc->rows == 0 || desc->cols == 0)
                return WH_ERR_SHAPE;
            if (!var_mode(desc->fmt, desc->rate, vmode, vparam))
                return WH_ERR_FORMAT;
            if (nbytes < var_index_bytes(desc->rows, desc->cols) + 16 || nbytes % 4)
                return WH_ERR_FORMAT;
            need = nbytes;
        } else {
            wh_status st = storage_bytes(*desc, need);
            if (st != WH_OK)
                return st;
            if (nbytes != need)
                return WH_ERR_FORMAT;
        }
        Matrix m{};
        m.desc = *desc;
        m.nbytes = need;
        if (where == WH_DEVICE) {
            if (!aligned(bytes, 16))
                return WH_ERR_INVALID;
            m.dptr = const_cast<void*>(bytes);
            m.owned = false;
        } else {
            void* d = nullptr;
            hipError_t e = hipMalloc(&d, need);
            if (e != hipSuccess)
                return device_error(ctx, e);
            e = hipMemcpy(d, bytes, need, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(d);
                return device_error(ctx, e);
            }
            m.dptr = d;
            m.owned = true;
        }
        std::lock_guard<std::mutex> lk(ctx->mu);
        const wh_mat id = ctx->next_id++;
        ctx->mats.emplace(id, m);
        *out = id;
        return WH_OK;
    } catch (const std::bad_alloc&) {
        return WH_ERR_NOMEM;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_unload(wh_ctx* ctx, wh_mat m)
{
    WH_GUARD(ctx);
    try {
        Matrix mat;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto it = ctx->mats.find(m);
            if (it == ctx->mats.end())
                return WH_ERR_NOT_FOUND;
            mat = it->second;
            ctx->mats.erase(it);
        }
        // the serving loop's graphs read the matrix: finish and drop them
        serve_forget(ctx, m);
        if (mat.owned) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess)
                return device_error(ctx, e);
            (void)hipFree(mat.dptr);
        }
        return WH_OK;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_gemv(wh_ctx* ctx, wh_mat m, const float* d_u, float* d_y, uint32_t row_begin, uint32_t row_end,
                  uint32_t flags, void* stream)
{
    WH_GUARD(ctx);
    if (!d_u || !d_y || !aligned(d_u, 16))
        return WH_ERR_INVALID;
    if (flags & ~(WH_ACC_FP64 | WH_ACC_TWOSUM | WH_PAPER_MP))
        return WH_ERR_INVALID;
    if ((flags & WH_ACC_FP64) && (flags & WH_ACC_TWOSUM))
        return WH_ERR_INVALID;
    try {
        Matrix mat;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            Matrix* p = find_matrix(ctx, m);
            if (!p)
                return WH_ERR_NOT_FOUND;
            mat = *p;
        }
        if (row_begin > row_end || row_end > mat.desc.rows)
            return WH_ERR_SHAPE;
        // block-scaled FP8 works on whole 4 x 4 tiles: a range of block rows
        if (mat.desc.fmt == WH_FMT_FP8E4M3_BS4 && (row_begin % 4 || row_end % 4))
            return WH_ERR_SHAPE;
        if (row_begin == row_end)
            return WH_OK;
        const AccMode mode = (flags & WH_PAPER_MP)     ? AccMode::PaperMp
                             : (flags & WH_ACC_TWOSUM) ? AccMode::TwoSum
                                                       : AccMode::Fp64;
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (is_var_format(mat.desc.fmt)) {
            if (mode == AccMode::PaperMp)
                return WH_ERR_FORMAT;
            const size_t pn = var_partials(mat, row_begin, row_end);
            if (pn) {
                wh_status s2 = ensure_partials(ctx, pn, st);
                if (s2 != WH_OK)
                    return s2;
            }
            hipError_t e = var_gemv(mat, mode, d_u, d_y, row_begin, row_end, pn ? ctx->part : nullptr, st);
            return device_error(ctx, pn ? partials_release(ctx, st, e) : e);
        }
        if (mat.desc.fmt == WH_FMT_ZFP_FIXED_RATE) {
            const GemvPlan pl =
                whz_gemv_plan(mat.desc.rate, mat.desc.rows, mat.desc.cols, row_begin, row_end, ctx->num_cus, &ctx->gemv_tune);
            double* part = nullptr;
            if (pl.nslab > 1) {
                wh_status s2 = ensure_partials(ctx, (size_t)pl.nslab * pl.part_rows(), st);
                if (s2 != WH_OK)
                    return s2;
                part = ctx->part;
            }
            hipError_t e = whz_gemv(mat.desc.rate, pl, mode, mat.dptr, d_u, d_y, part, st);
            return device_error(ctx, part ? partials_release(ctx, st, e) : e);
        }
        return dense_gemv_dispatch(ctx, mat, mode, d_u, d_y, row_begin, row_end, st);
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_gemv_batched(wh_ctx* ctx, wh_mat m, const void* d_U, int u_dtype, uint32_t k, uint32_t ldu, float* d_Y,
                          uint32_t ldy, uint32_t flags, void* stream)
{
    WH_GUARD(ctx);
    if (!d_U || !d_Y || k == 0 || k > kMaxRhs || (u_dtype != WH_U_F32 && u_dtype != WH_U_BF16))
        return WH_ERR_INVALID;
    if (flags & ~(WH_ACC_FP64 | WH_ACC_TWOSUM | WH_PAPER_MP))
        return WH_ERR_INVALID;
    try {
        Matrix mat;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            Matrix* p = find_matrix(ctx, m);
            if (!p)
                return WH_ERR_NOT_FOUND;
            mat = *p;
        }
        if (mat.desc.fmt != WH_FMT_ZFP_FIXED_RATE)
            return WH_ERR_FORMAT;
        if (ldu < mat.desc.cols || ldy < mat.desc.rows)
            return WH_ERR_SHAPE;
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (k == 1 && u_dtype == WH_U_F32 && aligned(d_U, 16)) // one vector: the fused k = 1 kernel
            return wh_gemv(ctx, m, static_cast<const float*>(d_U), d_Y, 0, mat.desc.rows, flags, stream);
        if (flags & WH_PAPER_MP)
            return WH_ERR_INVALID; // Fig. 7 per-product sums exist for one vector only
        const MrhsPlan pl = whz_mrhs_plan(mat.desc.rows, mat.desc.cols, 0, mat.desc.rows, ctx->num_cus, k,
                                          u_dtype == WH_U_BF16, &ctx->gemv_tune);
        // slab partials and B^T U share the context's workspace
        wh_status s2 = ensure_partials(ctx, mrhs_workspace(pl, k).total, st);
        if (s2 != WH_OK)
            return s2;
        hipError_t e = whz_mrhs(mat.desc.rate, pl, mat.dptr, d_U, ldu, k, d_Y, ldy, ctx->part, st);
        return device_error(ctx, partials_release(ctx, st, e));
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_decode_debug(wh_ctx* ctx, wh_mat m, uint64_t block_begin, uint64_t nblocks, float* d_out, void* stream)
{
    WH_GUARD(ctx);
    if (!d_out || !aligned(d_out, 16))
        return WH_ERR_INVALID;
    try {
        Matrix mat;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            Matrix* p = find_matrix(ctx, m);
            if (!p)
                return WH_ERR_NOT_FOUND;
            mat = *p;
        }
        if (mat.desc.fmt != WH_FMT_ZFP_FIXED_RATE)
            return WH_ERR_FORMAT;
        const uint64_t nb = (uint64_t)((mat.desc.rows + 3) / 4) * ((mat.desc.cols + 3) / 4);
        if (block_begin > nb || nblocks > nb - block_begin)
            return WH_ERR_INVALID;
        if (nblocks == 0)
            return WH_OK;
        return device_error(ctx, whz_decode_blocks(mat.desc.rate, mat.dptr, block_begin, nblocks, d_out,
                                                   static_cast<hipStream_t>(stream)));
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_decode(wh_ctx* ctx, wh_mat m, float* d_out, void* stream)
{
    WH_GUARD(ctx);
    if (!d_out || !aligned(d_out, 16))
        return WH_ERR_INVALID;
    try {
        Matrix mat;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            Matrix* p = find_matrix(ctx, m);
            if (!p)
                return WH_ERR_NOT_FOUND;
            mat = *p;
        }
        if (is_var_format(mat.desc.fmt))
            return device_error(ctx, var_decode(mat, d_out, static_cast<hipStream_t>(stream)));
        if (mat.desc.fmt != WH_FMT_ZFP_FIXED_RATE)
            return WH_ERR_FORMAT;
        return device_error(ctx, whz_decode_matrix(mat.desc.rate, mat.dptr, mat.desc.rows, mat.desc.cols, d_out,
                                                   static_cast<hipStream_t>(stream)));
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

wh_status wh_encode(wh_ctx* ctx, const float* d_M, uint32_t rows, uint32_t cols, uint32_t rate, void* d_stream,
                    uint32_t* d_bad, void* stream)
{
    WH_GUARD(ctx);
    if (!d_M || !d_stream || !aligned(d_M, 16) || !aligned(d_stream, 4))
        return WH_ERR_INVALID;
    if (rows == 0 || cols == 0)
        return WH_ERR_SHAPE;
    if (!whz_rate_supported(rate))
        return WH_ERR_FORMAT;
    try {
        return device_error(ctx, whz_encode(rate, d_M, rows, cols, d_stream, d_bad, static_cast<hipStream_t>(stream)));
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

} // extern "C"
