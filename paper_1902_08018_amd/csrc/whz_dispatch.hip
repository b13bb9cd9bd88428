// whz_dispatch.hip -- rate dispatch and launch planning for the WHZ1 kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wh_internal.hpp"

#define WH_FOR_EACH_NW(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(16)

namespace wh {

#define X(k)                                                                                                         \
    namespace nw##k {                                                                                                \
    hipError_t decode_blocks(const void*, uint64_t, uint64_t, float*, hipStream_t);                                  \
    hipError_t decode_matrix(const void*, uint32_t, uint32_t, float*, hipStream_t);                                  \
    hipError_t encode(const float*, uint32_t, uint32_t, void*, uint32_t*, hipStream_t);                              \
    hipError_t gemv(const GemvPlan&, AccMode, const void*, const float*, float*, double*, hipStream_t);              \
    hipError_t mrhs(const MrhsPlan&, bool, const void*, const void*, uint32_t, uint32_t, float*, uint32_t, double*,     \
                    hipStream_t);                                                                                      \
    }
WH_FOR_EACH_NW(X)
#undef X

bool whz_rate_supported(uint32_t rate)
{
    if (rate % 2)
        return false;
    switch (rate / 2) {
#define X(nw) case nw:
        WH_FOR_EACH_NW(X)
#undef X
        return true;
    default:
        return false;
    }
}

hipError_t whz_decode_blocks(uint32_t rate, const void* stream, uint64_t b0, uint64_t n, float* out, hipStream_t st)
{
    switch (rate / 2) {
#define X(k)                                                                                                         \
    case k:                                                                                                          \
        return nw##k::decode_blocks(stream, b0, n, out, st);
        WH_FOR_EACH_NW(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t whz_decode_matrix(uint32_t rate, const void* stream, uint32_t rows, uint32_t cols, float* out,
                             hipStream_t st)
{
    switch (rate / 2) {
#define X(k)                                                                                                         \
    case k:                                                                                                          \
        return nw##k::decode_matrix(stream, rows, cols, out, st);
        WH_FOR_EACH_NW(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t whz_encode(uint32_t rate, const float* M, uint32_t rows, uint32_t cols, void* stream, uint32_t* bad,
                      hipStream_t st)
{
    switch (rate / 2) {
#define X(k)                                                                                                         \
    case k:                                                                                                          \
        return nw##k::encode(M, rows, cols, stream, bad, st);
        WH_FOR_EACH_NW(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

GemvPlan whz_gemv_plan(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus, uint32_t lanes)
{
    (void)rows;
    const uint32_t kThreads = lanes;
    GemvPlan pl{};
    pl.nbc = cols / 4;
    pl.bi_begin = row_begin / 4;
    pl.bi_end = row_end / 4;
    const uint32_t nbr = pl.bi_end - pl.bi_begin;
    pl.ntiles = (nbr + kGemvTileRows - 1) / kGemvTileRows;
    // enough workgroups to fill the chip several times over
    const uint64_t want = (uint64_t)(num_cus > 0 ? num_cus : 256) * 8;
    const uint32_t max_slabs = (pl.nbc + kThreads - 1) / kThreads;
    uint32_t nslab = pl.ntiles ? (uint32_t)((want + pl.ntiles - 1) / pl.ntiles) : 1;
    if (nslab < 1)
        nslab = 1;
    if (nslab > max_slabs)
        nslab = max_slabs ? max_slabs : 1;
    uint32_t slab_bc = (pl.nbc + nslab - 1) / nslab;
    slab_bc = (slab_bc + kThreads - 1) / kThreads * kThreads;
    pl.slab_bc = slab_bc ? slab_bc : kThreads;
    pl.nslab = (pl.nbc + pl.slab_bc - 1) / pl.slab_bc;
    if (pl.nslab < 1)
        pl.nslab = 1;
    return pl;
}

hipError_t whz_gemv(uint32_t rate, const GemvPlan& pl, AccMode mode, const void* stream, const float* u, float* y,
                    double* part, hipStream_t st)
{
    if (pl.ntiles == 0)
        return hipSuccess;
    switch (rate / 2) {
#define X(k)                                                                                                         \
    case k:                                                                                                          \
        return nw##k::gemv(pl, mode, stream, u, y, part, st);
        WH_FOR_EACH_NW(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

MrhsPlan whz_mrhs_plan(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus)
{
    (void)rows;
    MrhsPlan pl{};
    pl.nbc = cols / 4;
    pl.bi_begin = row_begin / 4;
    pl.bi_end = row_end / 4;
    const uint32_t nbr = pl.bi_end - pl.bi_begin;
    pl.ntiles = (nbr + kMrhsTileBlockRows - 1) / kMrhsTileBlockRows;
    // two 8-wave workgroups are resident per CU: one full round of them;
    // more column slabs would only add FP64 partials (slabs x k x rows)
    const uint64_t want = (uint64_t)(num_cus > 0 ? num_cus : 256) * 2;
    const uint32_t max_slabs = (pl.nbc + 15) / 16;
    uint32_t nslab = pl.ntiles ? (uint32_t)((want + pl.ntiles - 1) / pl.ntiles) : 1;
    if (nslab < 1)
        nslab = 1;
    if (nslab > max_slabs)
        nslab = max_slabs ? max_slabs : 1;
    uint32_t slab_bc = (pl.nbc + nslab - 1) / nslab;
    slab_bc = (slab_bc + 15) / 16 * 16;
    pl.slab_bc = slab_bc ? slab_bc : 16;
    pl.nslab = (pl.nbc + pl.slab_bc - 1) / pl.slab_bc;
    if (pl.nslab < 1)
        pl.nslab = 1;
    return pl;
}

hipError_t whz_mrhs(uint32_t rate, const MrhsPlan& pl, bool bf16, const void* stream, const void* U, uint32_t ldu,
                    uint32_t k, float* Y, uint32_t ldy, double* part, hipStream_t st)
{
    if (pl.ntiles == 0)
        return hipSuccess;
    switch (rate / 2) {
#define X(kw)                                                                                                        \
    case kw:                                                                                                         \
        return nw##kw::mrhs(pl, bf16, stream, U, ldu, k, Y, ldy, part, st);
        WH_FOR_EACH_NW(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace wh
