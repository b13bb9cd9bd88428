// thermal.hip -- the thermal step of the model (Sec. 2.1, Eq. 1):
//
//     T_{k+1} = A T_k + B u_k,   A sparse (CSR), B diagonal,
//
// evaluated every millisecond (light and dark stages) on about 3.7e5
// temperatures before the deformation GEMV.  One lane per row: the row's
// products and b_i u_i are summed in FP64 (the kernel is bound by HBM, so the
// wide arithmetic costs nothing) and the state is stored as FP32.  Per row the
// kernel moves its CSR entries (8 B each), its row pointer, b_i, u_i, T_i and
// the new T_i (the gathered neighbours of a mesh come from cache).
#include <hip/hip_runtime.h>

#include "../../include/wh.h"
#include "wh_ctx.hpp"
#include "wh_internal.hpp"

namespace wh {
namespace {

constexpr int kThermalThreads = 256;

__global__ void __launch_bounds__(kThermalThreads) thermal_step_kernel(
    uint32_t n, uint32_t nnz, const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ col,
    const float* __restrict__ val, const float* __restrict__ b, const float* __restrict__ T,
    const float* __restrict__ u, float* __restrict__ T_next)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThermalThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThermalThreads + threadIdx.x; i < n; i += stride) {
        // entries outside [0, nnz) and columns outside [0, n) are skipped: a
        // malformed matrix gives wrong values, never a stray access
        const uint32_t p0 = row_ptr[i] < nnz ? row_ptr[i] : nnz;
        const uint32_t p1 = row_ptr[i + 1] < nnz ? row_ptr[i + 1] : nnz;
        double s = 0.0;
        for (uint32_t p = p0; p < p1; ++p) {
            const uint32_t j = col[p];
            if (j < n)
                s = __builtin_fma((double)val[p], (double)T[j], s);
        }
        s = __builtin_fma((double)b[i], (double)u[i], s);
        T_next[i] = (float)s;
    }
}

unsigned thermal_grid(uint32_t n)
{
    const uint64_t g = ((uint64_t)n + kThermalThreads - 1) / kThermalThreads;
    return (unsigned)(g < (1u << 20) ? (g ? g : 1) : (1u << 20));
}

} // namespace
} // namespace wh

using namespace wh;

extern "C" wh_status wh_thermal_step(wh_ctx* ctx, uint32_t n, uint32_t nnz, const uint32_t* d_row_ptr,
                                     const uint32_t* d_col, const float* d_val, const float* d_b, const float* d_T,
                                     const float* d_u, float* d_T_next, void* stream)
{
    WH_GUARD(ctx);
    if (!d_row_ptr || !d_b || !d_T || !d_u || !d_T_next || (nnz && (!d_col || !d_val)))
        return WH_ERR_INVALID;
    if (d_T == d_T_next)
        return WH_ERR_INVALID; // every row reads its neighbours' old values
    if (n == 0)
        return WH_OK;
    hipLaunchKernelGGL(thermal_step_kernel, dim3(thermal_grid(n)), dim3(kThermalThreads), 0,
                       static_cast<hipStream_t>(stream), n, nnz, d_row_ptr, d_col, d_val, d_b, d_T, d_u, d_T_next);
    return device_error(ctx, hipGetLastError());
}

extern "C" wh_status wh_thermal_run(wh_ctx* ctx, uint32_t n, uint32_t nnz, const uint32_t* d_row_ptr,
                                    const uint32_t* d_col, const float* d_val, const float* d_b, float* d_T,
                                    const float* d_U, uint64_t ldu, uint32_t steps, float* d_work, void* stream)
{
    WH_GUARD(ctx);
    if (!d_row_ptr || !d_b || !d_T || !d_work || (steps && !d_U) || (nnz && (!d_col || !d_val)))
        return WH_ERR_INVALID;
    if (d_T == d_work || ldu < n)
        return WH_ERR_INVALID;
    if (n == 0 || steps == 0)
        return WH_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // ping-pong between d_T and d_work; an odd count ends with a copy back
    float* cur = d_T;
    float* nxt = d_work;
    for (uint32_t k = 0; k < steps; ++k) {
        hipLaunchKernelGGL(thermal_step_kernel, dim3(thermal_grid(n)), dim3(kThermalThreads), 0, st, n, nnz,
                           d_row_ptr, d_col, d_val, d_b, cur, d_U + (uint64_t)k * ldu, nxt);
        float* t = cur;
        cur = nxt;
        nxt = t;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && cur != d_T)
        e = hipMemcpyAsync(d_T, cur, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st);
    return device_error(ctx, e);
}
