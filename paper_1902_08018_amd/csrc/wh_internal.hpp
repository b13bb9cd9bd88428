// wh_internal.hpp -- declarations shared by the libwh translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wh {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Accumulation of the cross-block row sums.
enum class AccMode { Fp64, TwoSum, PaperMp };

// Block-rows per workgroup tile of the fused GEMV, and its workgroup size.
constexpr int kGemvTileRows = 4;
constexpr uint32_t kGemvLanes = 512;

// Launch geometry of the fused GEMV over block-rows [bi_begin, bi_end).
struct GemvPlan {
    uint32_t nbc;      // block-columns (cols / 4)
    uint32_t bi_begin; // first block-row
    uint32_t bi_end;   // one past the last block-row
    uint32_t ntiles;   // row tiles of kGemvTileRows block-rows
    uint32_t slab_bc;  // block-columns per slab (multiple of 256)
    uint32_t nslab;    // column slabs; > 1 needs an FP64 partial workspace
};

// Launch geometry of the multi-RHS kernel: tiles of 16 block-rows x slabs of
// block-columns (multiples of 16).
typedef GemvPlan MrhsPlan;
constexpr uint32_t kMrhsTileBlockRows = 32;
constexpr uint32_t kMaxRhs = 64;

bool whz_rate_supported(uint32_t rate);
MrhsPlan whz_mrhs_plan(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus);
hipError_t whz_mrhs(uint32_t rate, const MrhsPlan& pl, bool bf16, const void* stream, const void* U, uint32_t ldu,
                    uint32_t k, float* Y, uint32_t ldy, double* part, hipStream_t st);
// lanes: workgroup size of the kernel the plan is for (slabs are multiples of it)
GemvPlan whz_gemv_plan(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus,
                       uint32_t lanes = kGemvLanes);
hipError_t whz_gemv(uint32_t rate, const GemvPlan& pl, AccMode mode, const void* stream, const float* u, float* y,
                    double* part, hipStream_t st);
hipError_t whz_decode_blocks(uint32_t rate, const void* stream, uint64_t b0, uint64_t n, float* out, hipStream_t st);
hipError_t whz_decode_matrix(uint32_t rate, const void* stream, uint32_t rows, uint32_t cols, float* out,
                             hipStream_t st);
hipError_t whz_encode(uint32_t rate, const float* M, uint32_t rows, uint32_t cols, void* stream, uint32_t* bad,
                      hipStream_t st);

} // namespace wh
