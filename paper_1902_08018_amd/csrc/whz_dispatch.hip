// whz_dispatch.hip -- rate dispatch and launch planning for the WHZ1 kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "wh_internal.hpp"

#define WH_FOR_EACH_NW(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(16)

namespace wh {

#define X(k)                                                                                                         \
    namespace nw##k {                                                                                                \
    hipError_t decode_blocks(const void*, uint64_t, uint64_t, float*, hipStream_t);                                  \
    hipError_t decode_matrix(const void*, uint32_t, uint32_t, float*, hipStream_t);                                  \
    hipError_t encode(const float*, uint32_t, uint32_t, void*, uint32_t*, hipStream_t);                              \
    hipError_t gemv(const GemvPlan&, AccMode, const void*, const float*, float*, double*, hipStream_t);              \
    hipError_t mrhs(const MrhsPlan&, const void*, const void*, uint32_t, uint32_t, float*, uint32_t, double*,           \
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

namespace {

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

GemvPlan range_plan(uint32_t cols, uint32_t row_begin, uint32_t row_end)
{
    GemvPlan pl{};
    pl.nbc = (cols + 3) / 4;
    pl.bi_begin = row_begin / 4;
    pl.bi_end = (row_end + 3) / 4;
    pl.cols = cols;
    pl.nrows = row_end - row_begin;
    pl.skip = row_begin & 3u;
    return pl;
}

// Slab width for `nslab` slabs of whole groups of `width` block columns;
// returns the slab count that width gives.
uint32_t set_slabs(GemvPlan& pl, uint32_t nslab, uint32_t width)
{
    uint32_t slab_bc = ceil_div(pl.nbc, nslab ? nslab : 1);
    slab_bc = ceil_div(slab_bc, width) * width;
    pl.slab_bc = slab_bc ? slab_bc : width;
    pl.nslab = ceil_div(pl.nbc, pl.slab_bc);
    if (pl.nslab < 1)
        pl.nslab = 1;
    return pl.nslab;
}

} // namespace

// Launch shape of the fused GEMV, chosen from sweeps of every shape over
// matrices from 378 x 256000 to 65536^2 on MI355X:
//  * 8 lanes per block row (14 % faster than 512 on 65536^2).  A wave then
//    decodes an 8 x 8 patch of blocks instead of 64 blocks of one row, and a
//    workgroup's slab of u is small and reused by its 64 block rows.  Wider
//    groups only where a tile of 512 / G block rows would be mostly empty
//    (few rows); narrower where a row has fewer than 8 block columns.
//  * One block row per group and tile.
//  * Column slabs of `iters` blocks per lane and row: about 2048 workgroups
//    (some three rounds of the 768 resident at once) with 3 to 16 blocks per
//    lane; past 2^27 blocks, about 8192 workgroups of up to 48 blocks per
//    lane, which keeps the FP64 partial sums small (the times differ by under
//    1 % there).
GemvPlan whz_gemv_plan(uint32_t rate, uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end,
                       int num_cus, const GemvTuning* tune)
{
    (void)rows;
    (void)num_cus;
    GemvPlan pl = range_plan(cols, row_begin, row_end);
    const uint32_t lanes = gemv_wg_lanes(rate), max_lg = gemv_max_lg(lanes);
    pl.lanes = lanes;
    const uint32_t nbr = pl.bi_end - pl.bi_begin;
    uint32_t lg = 3;
    while (lg > 2 && (1u << lg) > pl.nbc) // fewer block columns than lanes
        --lg;
    for (;;) { // the narrowest groups whose tiles are at least 90 % full
        const uint64_t tile = lanes >> lg;
        const uint64_t span = (uint64_t)ceil_div(nbr, tile) * tile;
        if (lg >= max_lg || 10 * (uint64_t)nbr >= 9 * span)
            break;
        ++lg;
    }
    uint32_t rpg = 1;
    if (tune && tune->lanes) {
        lg = 2;
        while ((1u << lg) < tune->lanes && lg < max_lg)
            ++lg;
    }
    if (tune && tune->rows && gemv_slots(lg, lanes) * 4 * tune->rows <= lanes && !gemv_one_tile_row(rate))
        rpg = tune->rows;
    pl.lg = lg;
    pl.rpg = rpg;
    pl.ntiles = ceil_div(nbr, (uint64_t)(lanes >> lg) * rpg);
    const uint32_t G = 1u << lg;
    const uint64_t blocks = (uint64_t)nbr * pl.nbc;
    const uint64_t per_wg = (uint64_t)lanes;
    uint64_t iters = std::min<uint64_t>(16, std::max<uint64_t>(3, (blocks + per_wg * 1024) / (per_wg * 2048)));
    if (blocks > (1ull << 27))
        iters = std::min<uint64_t>(48, blocks / (per_wg * 8192));
    uint32_t nslab = ceil_div(pl.nbc, (uint64_t)G * iters);
    if (tune && tune->slabs)
        nslab = tune->slabs;
    const uint32_t max_slabs = ceil_div(pl.nbc, G);
    set_slabs(pl, std::max(1u, std::min(nslab, max_slabs)), G);
    return pl;
}

GemvPlan block_slab_plan(uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus, uint32_t lanes,
                         uint32_t tile_rows)
{
    GemvPlan pl = range_plan(cols, row_begin, row_end);
    pl.lanes = lanes;
    const uint32_t nbr = pl.bi_end - pl.bi_begin;
    pl.ntiles = ceil_div(nbr, tile_rows);
    // enough workgroups to fill the chip several times over
    const uint64_t want = (uint64_t)(num_cus > 0 ? num_cus : 256) * 8;
    const uint32_t max_slabs = ceil_div(pl.nbc, lanes);
    uint32_t nslab = pl.ntiles ? ceil_div(want, pl.ntiles) : 1;
    if (nslab > max_slabs)
        nslab = max_slabs;
    set_slabs(pl, nslab ? nslab : 1, lanes);
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

MrhsPlan whz_mrhs_plan(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus, uint32_t k,
                       bool bf16, const GemvTuning* tune)
{
    (void)rows;
    const uint32_t slabs = tune ? tune->mrhs_slabs : 0;
    MrhsPlan pl{};
    const MrhsMath math = mrhs_math(k, bf16, tune && tune->mrhs_fp32);
    pl.math = (uint32_t)math;
    pl.nbc = (cols + 3) / 4;
    pl.bi_begin = row_begin / 4;
    pl.bi_end = (row_end + 3) / 4;
    pl.cols = cols;
    pl.nrows = row_end - row_begin;
    const uint32_t nbr = pl.bi_end - pl.bi_begin;
    const uint32_t tile_rows = 4u * (uint32_t)mrhs_waves((int)((k + 15) / 16), math);
    pl.ntiles = (nbr + tile_rows - 1) / tile_rows;
    // two workgroups are resident per CU; about two rounds of them, then the
    // slab count rounded up to a multiple of 8: on 65536^2 with up to 16
    // right-hand sides, 8 to 12 slabs (5 to 8 rounds) run 5.4 ms where 3
    // slabs (two rounds and two workgroups) take 6.2 ms and 5 to 7 take
    // 5.65 ms.  The L2 miss count is the same for 3 and 8 slabs (34.5 M and
    // 34.1 M): the gain is the shorter last round, not where B^T U is
    // cached.  Each column slab adds FP64 partials, slabs x k x rows
    const uint64_t want = (uint64_t)(num_cus > 0 ? num_cus : 256) * 4;
    const uint32_t max_slabs = (pl.nbc + 15) / 16;
    uint32_t nslab = pl.ntiles ? (uint32_t)((want + pl.ntiles - 1) / pl.ntiles) : 1;
    if (nslab < 1)
        nslab = 1;
    if (max_slabs >= 8)
        nslab = (nslab + 7) / 8 * 8;
    // the FP64 partials (slabs x k x rows) stay within 256 MiB: 8 slabs of up
    // to 64 right-hand sides over 65536 rows (at k = 64, 8 slabs take 7.27 ms
    // where 2 took 7.60); short row ranges (few tiles, which need the slabs to
    // fill the device) keep theirs
    const uint64_t per_slab = (uint64_t)std::max<uint32_t>(k, 1) * nbr * 4;
    const uint32_t cap = (uint32_t)std::max<uint64_t>(1, (32ull << 20) / std::max<uint64_t>(per_slab, 1));
    if (nslab > cap)
        nslab = cap;
    if (slabs)
        nslab = slabs;
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

hipError_t whz_mrhs(uint32_t rate, const MrhsPlan& pl, const void* stream, const void* U, uint32_t ldu, uint32_t k,
                    float* Y, uint32_t ldy, double* part, hipStream_t st)
{
    if (pl.ntiles == 0)
        return hipSuccess;
    switch (rate / 2) {
#define X(kw)                                                                                                        \
    case kw:                                                                                                         \
        return nw##kw::mrhs(pl, stream, U, ldu, k, Y, ldy, part, st);
        WH_FOR_EACH_NW(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace wh
