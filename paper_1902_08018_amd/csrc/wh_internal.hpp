// wh_internal.hpp -- declarations shared by the libwh translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wh {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Accumulation of the cross-block row sums.
enum class AccMode { Fp64, TwoSum, PaperMp };

// Workgroup size of the fused GEMV: 1024 lanes up to 16 bits/value, 768
// above.  Two workgroups share a CU: 32 waves at 1024 lanes, in 64 VGPRs
// each (the launch bounds ask for that), or 24 at 768 lanes, where a lane
// stages 13 or more words of LDS and two 1024-lane workgroups would not fit.
// The most lanes a group spans (512; 256 for 768, the largest power of two
// dividing it); the most block rows one lane group takes per tile.  The LDS
// doubles that hold the groups' row sums (slots x 4 x rows per group: one
// slot per wave, or per group of fewer than 64 lanes) are as many as the
// workgroup's lanes.
constexpr uint32_t kGemvLanes = 512;
constexpr uint32_t gemv_wg_lanes(uint32_t rate) { return rate <= 16 ? 1024u : 768u; }
// LDS of one workgroup when two share a CU
constexpr uint32_t kLdsPerWorkgroupOfTwo = 160u * 1024u / 2u;
// from 14 bits/value the row sums share the staging rows: one tile row
constexpr bool gemv_one_tile_row(uint32_t rate) { return rate >= 14 && rate <= 16; }
constexpr uint32_t gemv_max_lg(uint32_t lanes) { return lanes == 768u ? 8u : 9u; }
constexpr int kGemvMaxRowsPerGroup = 4;
constexpr uint32_t gemv_slots(uint32_t lg, uint32_t lanes) { return lg >= 6 ? lanes / 64 : lanes >> lg; }

// Launch geometry of the fused GEMV over rows [row_begin, row_end), i.e.
// block-rows [bi_begin, bi_end).  The `lanes` lanes of a workgroup form groups
// of 2^lg; each group sweeps one block row's slab of block columns, and a tile
// is (lanes >> lg) groups x rpg block rows.  A matrix whose sides are not multiples
// of 4 ends in partial blocks: the stream codes them edge-padded, u is taken as
// zero past the last column, and rows outside the range are not written.
struct GemvPlan {
    uint32_t nbc;      // block-columns (ceil(cols / 4))
    uint32_t bi_begin; // first block-row (row_begin / 4)
    uint32_t bi_end;   // one past the last block-row (ceil(row_end / 4))
    uint32_t ntiles;   // row tiles
    uint32_t slab_bc;  // block-columns per slab (a multiple of the group width)
    uint32_t nslab;    // column slabs; > 1 needs an FP64 partial workspace
    uint32_t cols;     // matrix columns
    uint32_t nrows;    // rows written: row_end - row_begin
    uint32_t lg;       // log2 of the lanes per group (2 .. 9)
    uint32_t rpg;      // block rows per group and tile (1 .. kGemvMaxRowsPerGroup)
    uint32_t skip;     // row_begin % 4: rows of the first block row before the range
    uint32_t lanes;    // workgroup lanes (gemv_wg_lanes of the rate)
    uint32_t math;     // multi-RHS plans: the contraction (MrhsMath)
    // FP64 partials per slab and right-hand side: the range's block-rows
    uint32_t part_rows() const { return (bi_end - bi_begin) * 4; }
};

// Fixed launch shape for the fused GEMV (tuning and tests): zero fields are
// left to the planner.
struct GemvTuning {
    uint32_t lanes = 0; // lanes per group: 4, 8, ..., 512
    uint32_t rows = 0;  // block rows per group and tile: 1 .. kGemvMaxRowsPerGroup
    uint32_t slabs = 0; // column slabs (at most one per group width of block columns)
    uint32_t mrhs_slabs = 0; // column slabs of the multi-RHS kernel
    uint32_t mrhs_fp32 = 0;  // 1: FP32 U always on the 16x16x4 FP32 MFMA (no three-part split, no 4x4x1)
};

// Launch geometry of the multi-RHS kernel: tiles of 4 block-rows per wave x
// slabs of block-columns (multiples of 16).
typedef GemvPlan MrhsPlan;
// How it contracts: FP32 U on the FP32 MFMA; BF16 U on the BF16 MFMA; or FP32
// U and the FP32 coefficients each split into three BF16 parts, whose six
// significant products go to the BF16 MFMA (X6: from 17 right-hand sides up,
// where the FP32 MFMA's time, which does not overlap the decoder's VALU work,
// exceeds the split's VALU cost).
// F32: v_mfma_f32_16x16x4f32 over groups of 16 right-hand sides; F32N: up
// to kMrhsNarrowMax right-hand sides on v_mfma_f32_4x4x1f32 (16 blocks);
// Bf16: BF16 U; X6: FP32 U as three BF16 parts.
enum class MrhsMath : uint32_t { F32 = 0, Bf16 = 1, X6 = 2, F32N = 3 };
constexpr uint32_t kMrhsNarrowMax = 4;
inline MrhsMath mrhs_math(uint32_t k, bool bf16, bool force_fp32)
{
    if (bf16)
        return MrhsMath::Bf16;
    if (force_fp32)
        return MrhsMath::F32;
    return k > 16 ? MrhsMath::X6 : (k <= kMrhsNarrowMax ? MrhsMath::F32N : MrhsMath::F32);
}
// Waves per workgroup for NT groups of 16 right-hand sides: 16 up to 16
// right-hand sides, 8 above (two workgroups per CU in LDS and registers).
constexpr int mrhs_waves(int nt, MrhsMath m) { return m == MrhsMath::X6 ? 8 : (nt == 1 ? 16 : 8); }
constexpr uint32_t kMrhsMaxTileBlockRows = 64;
constexpr uint32_t kMaxRhs = 64;

// The multi-RHS workspace, in doubles: FP64 slab partials [nslab][k][rows]
// (only when the plan splits the columns), then, from btu_offset (a whole
// number of 256-byte lines in), B^T U for every block column rounded up to
// 16 and every group of 16 right-hand sides (FP32, BF16, or three BF16
// parts: 4, 2 or 6 bytes per value).
struct MrhsWorkspace {
    size_t btu_offset;
    size_t total;
};
inline MrhsWorkspace mrhs_workspace(const MrhsPlan& pl, uint32_t k)
{
    const size_t part = pl.nslab > 1 ? (size_t)pl.nslab * k * pl.part_rows() : 0;
    const size_t off = (part + 31) / 32 * 32;
    const size_t nbc16 = ((size_t)pl.nbc + 15) / 16 * 16;
    const size_t nt = (k + 15) / 16;
    const MrhsMath m = (MrhsMath)pl.math;
    const size_t btu_bytes = nbc16 * nt * 64 * (m == MrhsMath::Bf16 ? 2 : m == MrhsMath::X6 ? 6 : 4);
    return MrhsWorkspace{off, off + (btu_bytes + 7) / 8};
}

bool whz_rate_supported(uint32_t rate);
// for k right-hand sides, FP32 or BF16 U; `tune` (may be null) can fix the
// column slab count and keep FP32 U on the FP32 MFMA
MrhsPlan whz_mrhs_plan(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus, uint32_t k,
                       bool bf16, const GemvTuning* tune = nullptr);
// `ws`: mrhs_workspace(pl, k).total doubles of device memory; U is BF16 when
// the plan's math is MrhsMath::Bf16, else FP32
hipError_t whz_mrhs(uint32_t rate, const MrhsPlan& pl, const void* stream, const void* U, uint32_t ldu, uint32_t k,
                    float* Y, uint32_t ldy, double* part, hipStream_t st);
GemvPlan whz_gemv_plan(uint32_t rate, uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end,
                       int num_cus, const GemvTuning* tune = nullptr);
// Slabs of block columns for a kernel whose `lanes` lanes sweep each block row
// of a tile of `tile_rows` block rows together (the block-scaled FP8 GEMV).
GemvPlan block_slab_plan(uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus, uint32_t lanes,
                         uint32_t tile_rows);
hipError_t whz_gemv(uint32_t rate, const GemvPlan& pl, AccMode mode, const void* stream, const float* u, float* y,
                    double* part, hipStream_t st);
hipError_t whz_decode_blocks(uint32_t rate, const void* stream, uint64_t b0, uint64_t n, float* out, hipStream_t st);
hipError_t whz_decode_matrix(uint32_t rate, const void* stream, uint32_t rows, uint32_t cols, float* out,
                             hipStream_t st);
hipError_t whz_encode(uint32_t rate, const float* M, uint32_t rows, uint32_t cols, void* stream, uint32_t* bad,
                      hipStream_t st);

} // namespace wh
