// mrhs_kernels.hip -- multi-right-hand-side GEMV (wh_gemv_batched).
#include <hip/hip_runtime.h>

#include "wh_ctx.hpp"

extern "C" wh_status wh_gemv_batched(wh_ctx* ctx, wh_mat m, const void* d_U, int u_dtype, uint32_t k, uint32_t ldu,
                                     float* d_Y, uint32_t ldy, uint32_t flags, void* stream)
{
    (void)ctx; (void)m; (void)d_U; (void)u_dtype; (void)k; (void)ldu; (void)d_Y; (void)ldy; (void)flags; (void)stream;
    return WH_ERR_INVALID;
}
