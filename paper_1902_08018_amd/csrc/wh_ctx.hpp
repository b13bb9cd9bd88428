// wh_ctx.hpp -- the library context (opaque wh_ctx of include/wh.h).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "../../include/wh.h"
#include "wh_internal.hpp"

namespace wh {

struct Matrix {
    wh_matrix_desc desc;
    void* dptr;      // device storage (stream, dense values, or codes+scales)
    uint64_t nbytes; // == storage bytes of desc
    bool owned;      // copied in by the library (WH_HOST)
};

struct Server;   // serving loop state (serve.hip)
struct HostPipe; // copy stream and staging of wh_gemv_host (host_stream.hip)

// wh_gemv_host: staging buffers used in turn, and the default chunk of
// compressed bytes per copy.
constexpr int kPipeBuffers = 2;
constexpr uint64_t kPipeChunkBytes = 32ull << 20;
// Waits for the pipe's copies and frees it (wh_destroy).
void host_pipe_free(wh_ctx* ctx);

// Variable-rate WHZ1 (fixed precision / fixed accuracy), whz_var.hip.
inline bool is_var_format(int fmt) { return fmt == WH_FMT_ZFP_FIXED_PRECISION || fmt == WH_FMT_ZFP_FIXED_ACCURACY; }
bool var_mode(int fmt, uint32_t rate, int& mode, int& param);
uint32_t var_groups(uint32_t cols);
uint64_t var_index_bytes(uint32_t rows, uint32_t cols);
hipError_t var_decode(const Matrix& m, float* out, hipStream_t st);
size_t var_partials(const Matrix& m, uint32_t row_begin, uint32_t row_end);
hipError_t var_gemv(const Matrix& m, AccMode acc, const float* u, float* y, uint32_t row_begin, uint32_t row_end,
                    double* part, hipStream_t st);

wh_status device_error(wh_ctx* ctx, hipError_t e);
// The context's FP64 slab-partials workspace, shared by every call that
// splits columns: grow it to `count` doubles, and make `st` wait until the
// previous user's work on the device is done (on whatever stream it ran).
// The user then calls partials_release after its launches.  Returns
// WH_ERR_INVALID while `st` is being captured into a graph: a later call may
// regrow (free) the workspace that the graph would keep using.
wh_status ensure_partials(wh_ctx* ctx, size_t count, hipStream_t st);
hipError_t partials_release(wh_ctx* ctx, hipStream_t st, hipError_t e);
Matrix* find_matrix(wh_ctx* ctx, wh_mat m);
bool aligned(const void* p, uintptr_t a);

// Dense-storage GEMV (FP32 / FP16 / BF16 / FP8 block-scaled), dense_kernels.hip.
wh_status dense_gemv_dispatch(wh_ctx* ctx, const Matrix& mat, AccMode mode, const float* d_u, float* d_y,
                              uint32_t row_begin, uint32_t row_end, hipStream_t st);

// With `device` current, find the device address of wh_gemv_noalloc's
// scratch array on it (once per device); wh_create calls it.
wh_status noalloc_init(int device);

void serve_shutdown(wh_ctx* ctx);
// Drop the serving state of matrix m (after its batches in flight finish;
// its queued requests complete with WH_ERR_NOT_FOUND).
void serve_forget(wh_ctx* ctx, wh_mat m);

} // namespace wh

struct wh_ctx {
    int device = 0;
    int num_cus = 256;
    wh::GemvTuning gemv_tune; // launch-shape overrides read at wh_create
    uint64_t serve_chunk_values = 1ull << 28; // values per serving launch (WH_SERVE_CHUNK_VALUES)
    uint32_t serve_shed = 0; // shed when the queue head waited this many deadlines (WH_SERVE_SHED; 0 = never)
    double serve_pace = 4.0; // a late scan's chunk times per launch while other work waits (WH_SERVE_PACE)
    double serve_margin_ns = 1e6; // a held request's margin before its deadline (WH_SERVE_MARGIN_US)
    uint64_t budget = 0;
    std::mutex mu; // guards mats / next_id
    std::unordered_map<wh_mat, wh::Matrix> mats;
    wh_mat next_id = 1;
    double* part = nullptr; // FP64 slab partials
    size_t part_cap = 0;
    hipEvent_t part_ev = nullptr; // recorded after each user of `part`
    std::atomic<bool> failed{false};
    wh::Server* server = nullptr; // owned; freed by serve_shutdown
    wh::HostPipe* pipe = nullptr;  // owned; freed by host_pipe_free
};

// Entry-point prologue: a live context whose device is current.
#define WH_GUARD(ctx)                                                                                               \
    do {                                                                                                             \
        if (!(ctx))                                                                                                  \
            return WH_ERR_INVALID;                                                                                   \
        if ((ctx)->failed.load())                                                                                    \
            return WH_ERR_DEVICE;                                                                                    \
        if (hipSetDevice((ctx)->device) != hipSuccess)                                                               \
            return WH_ERR_DEVICE;                                                                                    \
    } while (0)
