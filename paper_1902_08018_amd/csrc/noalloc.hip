// noalloc.hip -- the fused compressed GEMV for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops that forbid
// hipMalloc): wh_gemv_noalloc of include/wh.h.
//
// The only device memory the fused GEMV needs beyond its inputs and outputs
// is the FP64 slab-partials workspace (one double per column slab and row of
// the range).  Here it is a file-scope device array, `scratch`, of a fixed
// size.  Each GPU the library runs on holds its own copy of the array, from
// the first context created on it until the process ends.
//
// Host code never passes the array's name to a kernel: on the host that name
// is a stand-in, not a device address.  wh_create looks up the array's device
// address once per device (with that device current) and keeps it here; the
// entry point hands that address to the kernels.
//
// Every call on one GPU shares that GPU's array.  Calls whose work overlaps
// on the device (on different streams, or from different contexts) race on
// it; calls ordered on one stream do not.  Nothing in the array needs to start
// at zero: the GEMV writes every partial of its plan before the reduction
// reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/wh.h"
#include "wh_ctx.hpp"
#include "wh_internal.hpp"

namespace wh {

constexpr uint64_t kScratchDoubles = WH_NOALLOC_SCRATCH_BYTES / sizeof(double);
static_assert(WH_NOALLOC_SCRATCH_BYTES % 256 == 0, "the scratch array is whole 256-byte lines");

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

} // namespace

// With `device` current: look up this device's copy of the scratch array
// (once per device and process).
wh_status noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return WH_ERR_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device])
        return WH_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return WH_ERR_DEVICE;
    }
    g_scratch[device] = static_cast<double*>(p);
    return WH_OK;
}

namespace {

double* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_scratch[device];
}

} // namespace
} // namespace wh

using namespace wh;

extern "C" wh_status wh_gemv_noalloc(wh_ctx* ctx, wh_mat m, const float* d_u, float* d_y, uint32_t row_begin,
                                     uint32_t row_end, uint32_t flags, void* stream)
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
        if (mat.desc.fmt != WH_FMT_ZFP_FIXED_RATE)
            return WH_ERR_FORMAT;
        if (row_begin > row_end || row_end > mat.desc.rows)
            return WH_ERR_SHAPE;
        if (row_begin == row_end)
            return WH_OK;
        const AccMode mode = (flags & WH_PAPER_MP)     ? AccMode::PaperMp
                             : (flags & WH_ACC_TWOSUM) ? AccMode::TwoSum
                                                       : AccMode::Fp64;
        // the same launch plan as wh_gemv, so the two give the same y
        const GemvPlan pl =
            whz_gemv_plan(mat.desc.rate, mat.desc.rows, mat.desc.cols, row_begin, row_end, ctx->num_cus, &ctx->gemv_tune);
        double* part = nullptr;
        if (pl.nslab > 1) {
            if ((uint64_t)pl.nslab * pl.part_rows() > kScratchDoubles)
                return WH_ERR_SCRATCH;
            part = scratch_of(ctx->device);
            if (!part) // wh_create found no scratch array on this device
                return WH_ERR_DEVICE;
        }
        return device_error(ctx, whz_gemv(mat.desc.rate, pl, mode, mat.dptr, d_u, d_y, part,
                                          static_cast<hipStream_t>(stream)));
    } catch (...) {
        return WH_ERR_INVALID;
    }
}
