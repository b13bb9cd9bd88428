// whz_kernels.hip -- WHZ1 kernels for gfx950: decode probe, full decode,
// encoder, the fused decode + mixed-precision GEMV (k = 1) and the
// multi-right-hand-side product.
//
// Fused GEMV (the deformation product y = C.S of Eq. 2 over a zfp-compressed
// matrix, Sec. 4.3-4.4):
//   grid     one 512-lane workgroup per (row tile, column slab)
//   lanes    groups of 2^lg lanes (8 by default); a group sweeps one block
//            row's slab, each lane decoding one 4x4 block per step (its
//            words staged in LDS), so a wave works on an 8 x 8 patch of
//            blocks; a tile holds (512 / 2^lg) x rpg block rows
//   product  each block's coefficients against B^T u (FP32), its power-of-two
//            scale applied to the sum; B once per block row at the end; blocks
//            cut by the bit budget above plane 26 take the exact inverse lift
//   sums     FP32 within a block (4 products), then FP64 (or compensated
//            FP32) across blocks; shuffles within the group, LDS across
//            waves; one FP64 partial per row and slab
//   reduce   a second kernel adds the slab partials in FP64 and rounds once
//            to FP32 (skipped when there is a single slab)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "whz_device.hpp"
#include "wh_internal.hpp"

namespace wh {
namespace {

constexpr int kThreads = 256;

// The section table, built at compile time; copied to LDS by every workgroup.
__device__ const SectionTable g_section_table{};

template <int THREADS>
__device__ __forceinline__ void load_section_table(uint32_t* tab)
{
    for (int i = threadIdx.x; i < kSecEntries; i += THREADS)
        tab[i] = g_section_table.e[i];
    __syncthreads();
}

// Staged blocks live word-major in LDS: word q of the block of lane l is at
// lds[q * STRIDE + l] (STRIDE = the workgroup's lanes), so every lane-varying
// read of a wave touches 64 distinct banks.
// Stage one block (NW words at g) at lw = lds + lane.
template <int NW, int STRIDE>
__device__ __forceinline__ void stage_block(uint32_t* lw, const uint32_t* __restrict__ g, uint32_t (&w)[NW])
{
    if constexpr (NW % 4 == 0) {
        const u32x4* g4 = reinterpret_cast<const u32x4*>(g);
#pragma unroll
        for (int k = 0; k < NW / 4; ++k) {
            const u32x4 v = __builtin_nontemporal_load(g4 + k);
            w[4 * k] = v.x;
            w[4 * k + 1] = v.y;
            w[4 * k + 2] = v.z;
            w[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k)
            w[k] = g[k];
    }
#pragma unroll
    for (int k = 0; k < NW; ++k)
        lw[k * STRIDE] = w[k];
}

template <int NW, int STRIDE>
__device__ __forceinline__ void clear_pad(uint32_t* lw)
{
#pragma unroll
    for (int k = NW; k < kStagedWords<NW>; ++k)
        lw[k * STRIDE] = 0u;
}

// ------------------------------------------------------- decode kernels
template <int NW>
__global__ void __launch_bounds__(kThreads) decode_blocks_kernel(const uint32_t* __restrict__ stream, uint64_t b0,
                                                                 uint64_t nblocks, float* __restrict__ out)
{
    __shared__ uint32_t lds[kThreads * kStagedWords<NW>];
    __shared__ uint32_t tab[kSecEntries];
    uint32_t* row = lds + threadIdx.x;
    clear_pad<NW, kThreads>(row);
    load_section_table<kThreads>(tab);
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < nblocks; i += stride) {
        uint32_t w[NW];
        stage_block<NW, kThreads>(row, stream + (b0 + i) * NW, w);
        int emax;
        uint32_t iv[16];
        decode_block_ints<NW, kThreads>(row, tab, w[0], emax, iv);
        float4* o = reinterpret_cast<float4*>(out + 16 * i);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            o[r] = make_float4(__builtin_ldexpf((float)(int32_t)iv[4 * r], emax - 30),
                               __builtin_ldexpf((float)(int32_t)iv[4 * r + 1], emax - 30),
                               __builtin_ldexpf((float)(int32_t)iv[4 * r + 2], emax - 30),
                               __builtin_ldexpf((float)(int32_t)iv[4 * r + 3], emax - 30));
    }
}

// Whole matrix into row-major FP32 (rows x cols).  A wave decodes an 8 x 8
// patch of blocks (lane l: block row 8i + l / 8, block column 8j + l % 8):
// the lanes run the bit planes in lockstep, and neighbouring blocks need more
// alike numbers of planes and lookups than 64 blocks along one row.  Wide
// workgroups share one copy of the section table among more waves.
template <int NW>
constexpr int kDecThreads = NW <= 8 ? 1024 : 512;

template <int NW>
__global__ void __launch_bounds__(kDecThreads<NW>) decode_matrix_kernel(const uint32_t* __restrict__ stream,
                                                                        uint32_t nbr, uint32_t nbc, uint32_t npc,
                                                                        uint64_t npatch, uint32_t rows, uint32_t cols,
                                                                        float* __restrict__ out)
{
    constexpr int T = kDecThreads<NW>;
    constexpr uint32_t kWaves = T / 64;
    __shared__ uint32_t lds[T * kStagedWords<NW>];
    __shared__ uint32_t tab[kSecEntries];
    uint32_t* row = lds + threadIdx.x;
    clear_pad<NW, T>(row);
    load_section_table<T>(tab);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    const uint32_t lane = threadIdx.x % 64u;
    const uint64_t stride = (uint64_t)gridDim.x * kWaves;
    for (uint64_t p = (uint64_t)blockIdx.x * kWaves + wave; p < npatch; p += stride) {
        const uint64_t bi = (p / npc) * 8u + lane / 8u, bj = (p % npc) * 8u + lane % 8u;
        if (bi >= nbr || bj >= nbc)
            continue;
        uint32_t w[NW];
        stage_block<NW, T>(row, stream + (bi * nbc + bj) * NW, w);
        int emax;
        uint32_t iv[16];
        decode_block_ints<NW, T>(row, tab, w[0], emax, iv);
        if ((cols & 3u) == 0 && 4 * bi + 3 < rows) { // a whole block on 16-byte aligned rows
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                f32x4 v;
                v.x = __builtin_ldexpf((float)(int32_t)iv[4 * r], emax - 30);
                v.y = __builtin_ldexpf((float)(int32_t)iv[4 * r + 1], emax - 30);
                v.z = __builtin_ldexpf((float)(int32_t)iv[4 * r + 2], emax - 30);
                v.w = __builtin_ldexpf((float)(int32_t)iv[4 * r + 3], emax - 30);
                __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(out + (4 * bi + r) * cols + 4 * bj));
            }
        } else { // the values of the block inside the matrix (the padding is dropped)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (4 * bi + r < rows && 4 * bj + c < cols)
                        out[(4 * bi + r) * cols + 4 * bj + c] = __builtin_ldexpf((float)(int32_t)iv[4 * r + c], emax - 30);
        }
    }
}

// ---------------------------------------------------------------- encoder
template <int NW>
__global__ void __launch_bounds__(kThreads) encode_kernel(const float* __restrict__ M, uint32_t nbc, uint32_t rows,
                                                          uint32_t cols, uint64_t nblocks, uint32_t* __restrict__ stream,
                                                          uint32_t* __restrict__ bad)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < nblocks; b += stride) {
        const uint64_t bi = b / nbc, bj = b % nbc;
        float f[16];
        if ((cols & 3u) == 0 && 4 * bi + 3 < rows) { // a whole block on 16-byte aligned rows
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float4 v = *reinterpret_cast<const float4*>(M + (4 * bi + r) * cols + 4 * bj);
                f[4 * r] = v.x;
                f[4 * r + 1] = v.y;
                f[4 * r + 2] = v.z;
                f[4 * r + 3] = v.w;
            }
        } else { // a partial block is completed by repeating the last row / column
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t i = 4 * bi + r < rows ? 4 * bi + r : rows - 1;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint64_t j = 4 * bj + c < cols ? 4 * bj + c : cols - 1;
                    f[4 * r + c] = M[i * cols + j];
                }
            }
        }
        uint32_t out[NW];
        const bool finite = encode_block<NW>(f, out);
        if (!finite && bad)
            atomicAdd(bad, 1u);
#pragma unroll
        for (int k = 0; k < NW; ++k)
            stream[b * NW + k] = out[k];
    }
}

// ------------------------------------------------------------ fused GEMV
struct Fp64Acc {
    static constexpr bool kPerProduct = false;
    double s;
    __device__ __forceinline__ void zero() { s = 0.0; }
    __device__ __forceinline__ void add(float p) { s += (double)p; }
    __device__ __forceinline__ double value() const { return s; }
    __device__ __forceinline__ void merge_from_lane(int mask)
    {
        s += __shfl_xor(s, mask, 64);
    }
};

// The paper's mixed-precision reduction (Fig. 7): FP64 sum of FP32 products.
struct PaperMpAcc : Fp64Acc {
    static constexpr bool kPerProduct = true;
};

// Compensated FP32 accumulator (Knuth TwoSum: hi + lo carries the exact sum
// of the added FP32 values up to the rounding of lo).
struct TwoSumAcc {
    static constexpr bool kPerProduct = false;
    float hi, lo;
    __device__ __forceinline__ void zero() { hi = lo = 0.0f; }
    __device__ __forceinline__ void add(float p)
    {
        const float s = hi + p;
        const float bp = s - hi;
        const float e = (hi - (s - bp)) + (p - bp);
        hi = s;
        lo += e;
    }
    __device__ __forceinline__ double value() const { return (double)hi + (double)lo; }
    __device__ __forceinline__ void merge_from_lane(int mask)
    {
        const float ohi = __shfl_xor(hi, mask, 64), olo = __shfl_xor(lo, mask, 64);
        add(ohi);
        lo += olo;
    }
};

// workgroup lanes of the fused GEMV for NW words per block (2 NW bits/value)
template <int NW>
constexpr int kGemvThreads = (int)gemv_wg_lanes(2 * NW);

// L = B^-1 = (1/16) [[4, 4, 4, 4], [5, 1, -1, -5], [-4, 4, 4, -4],
// [-2, 6, -6, 2]] (the forward lift's linear part) on (a, b, c, d).
__device__ __forceinline__ void lin_fwd(float a, float b, float c, float d, float& o0, float& o1, float& o2,
                                        float& o3)
{
    o0 = 0.25f * (a + b + c + d);
    o1 = 0.0625f * (5.0f * (a - d) + (b - c));
    o2 = 0.25f * ((b + c) - (a + d));
    o3 = 0.0625f * (2.0f * (d - a) + 6.0f * (b - c));
}

// A block whose bit budget ended above plane kSafeCutPlane: its exact row
// sums z = X u (X the decoded integers, through the integer inverse lift)
// replace the coefficient-space sums by L z, so that applying B to the row
// group's sums gives z back.
__device__ __forceinline__ void exact_block_sums(const uint32_t (&cf)[16], float4 uu, float (&v)[4])
{
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        x[i] = cf[i];
    inv_xform(x);
    float z[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        z[r] = (float)(int32_t)x[4 * r] * uu.x;
        z[r] = __builtin_fmaf((float)(int32_t)x[4 * r + 1], uu.y, z[r]);
        z[r] = __builtin_fmaf((float)(int32_t)x[4 * r + 2], uu.z, z[r]);
        z[r] = __builtin_fmaf((float)(int32_t)x[4 * r + 3], uu.w, z[r]);
    }
    lin_fwd(z[0], z[1], z[2], z[3], v[0], v[1], v[2], v[3]);
}

// The same for the multi-RHS tile: the block's scaled coefficients become
// L X L^T (X the exactly decoded integers), so that B (.) B^T gives X back.
__device__ __forceinline__ void exact_block_coeffs(const uint32_t (&cf)[16], int emax, float (&sc)[16])
{
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        x[i] = cf[i];
    inv_xform(x);
    float f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        f[i] = (float)(int32_t)x[i];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        lin_fwd(f[4 * r], f[4 * r + 1], f[4 * r + 2], f[4 * r + 3], f[4 * r], f[4 * r + 1], f[4 * r + 2],
                f[4 * r + 3]);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        lin_fwd(f[c], f[4 + c], f[8 + c], f[12 + c], f[c], f[4 + c], f[8 + c], f[12 + c]);
#pragma unroll
    for (int i = 0; i < 16; ++i)
        sc[i] = __builtin_ldexpf(f[i], emax - 30);
}

// The workgroup's lanes (1024, or 768 from 17 bits/value) form groups of
// 2^lg lanes (4 to 512).  A group sweeps a block row's slab of block columns,
// its lanes striding them; the workgroup's tile is (lanes >> lg) groups x rpg
// block rows, group g taking the tile's rows g, g + groups, ...  Square and
// tall matrices use groups of 8 lanes (a wave decodes an 8 x 8 patch of
// blocks); narrow ones (few block columns) use smaller groups, so that every
// lane has blocks to decode, and few block rows wider ones.  Output row i of
// the range is matrix row 4 * bi_begin + skip + i.
// two workgroups per CU: 1024-lane ones in 64 VGPRs (32 waves)
template <int NW>
constexpr int kGemvMinWaves = kGemvThreads<NW> == 1024 ? 8 : 6;
// From 14 bits/value a 1024-lane workgroup's staging rows and section table
// leave no room for its own row-sum doubles within two workgroups' LDS; the
// sums then go over the staging rows once every wave has decoded its blocks,
// which needs one tile row per group (the planner's choice there).
template <int NW>
constexpr bool kGemvSumsInStaging =
    kGemvThreads<NW> * (kStagedWords<NW> * 4 + 8) + kSecEntries * 4 > kLdsPerWorkgroupOfTwo;

template <int NW, typename Acc>
__global__ void __launch_bounds__(kGemvThreads<NW>, kGemvMinWaves<NW>) gemv_kernel(const uint32_t* __restrict__ stream,
                                                        const float* __restrict__ u, float* __restrict__ y,
                                                        double* __restrict__ part, uint32_t nbc, uint32_t bi_begin,
                                                        uint32_t bi_end, uint32_t slab_bc, uint32_t nslab,
                                                        uint32_t cols, uint32_t nrows, uint32_t lg, uint32_t rpg,
                                                        uint32_t skip)
{
    constexpr int THREADS = kGemvThreads<NW>;
    constexpr bool kShared = kGemvSumsInStaging<NW>;
    __shared__ __align__(16) uint32_t lds[THREADS * kStagedWords<NW>];
    __shared__ uint32_t tab[kSecEntries];
    // a group's four row sums per tile row: one slot per wave when a group
    // spans whole waves, else one per group (over the staging rows when they
    // must share its LDS)
    __shared__ double red_own[kShared ? 1 : THREADS];
    static_assert(!kShared || kStagedWords<NW> >= 2, "the row sums fit the staging rows");
    double* red = kShared ? reinterpret_cast<double*>(lds) : red_own;
    uint32_t* row = lds + threadIdx.x;
    clear_pad<NW, THREADS>(row);
    load_section_table<THREADS>(tab);

    const uint32_t G = 1u << lg, groups = (uint32_t)THREADS >> lg;
    const uint32_t grp = threadIdx.x >> lg, gl = threadIdx.x & (G - 1);
    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t bi0 = bi_begin + tile * groups * rpg;
    const uint32_t bc0 = slab * slab_bc;
    const uint32_t bc1 = bc0 + slab_bc < nbc ? bc0 + slab_bc : nbc;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool wide = lg >= 6; // a group spans whole waves
    const uint32_t slot = wide ? (uint32_t)wave : grp, slot_len = 4 * rpg;
    const bool leader = wide ? lane == 0 : gl == 0;
    const int first_mask = wide ? 32 : (int)(G >> 1);
    const float4* u4 = reinterpret_cast<const float4*>(u);
    // one tile row at a time (rolled loop: one copy of the decoder), so only
    // that row's four accumulators are live while blocks decode
#pragma unroll 1
    for (uint32_t t = 0; t < rpg; ++t) {
        const uint32_t bi = bi0 + t * groups + grp;
        // the same for every lane of the group; with the sums over the
        // staging rows (one tile row) every wave goes on to the barrier below
        if (!kShared && bi >= bi_end)
            break;
        Acc acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[r].zero();
        const uint32_t* srow = stream + (uint64_t)bi * nbc * NW;
        for (uint32_t bj = bc0 + gl; bi < bi_end && bj < bc1; bj += G) {
            float4 uu;
            if (4 * bj + 3 < cols) {
                uu = u4[bj];
            } else { // the partial last block column: u is zero past the last column
                const uint32_t j = 4 * bj;
                uu.x = u[j];
                uu.y = j + 1 < cols ? u[j + 1] : 0.0f;
                uu.z = j + 2 < cols ? u[j + 2] : 0.0f;
                uu.w = 0.0f;
            }
            uint32_t w[NW];
            stage_block<NW, THREADS>(row, srow + (uint64_t)bj * NW, w);
            int emax;
            uint32_t iv[16];
            if constexpr (Acc::kPerProduct) {
                // Fig. 7: each FP32 product of the decoded value and u is
                // added to the FP64 sum on its own
                decode_block_ints<NW, THREADS>(row, tab, w[0], emax, iv);
                const int k = emax - 30;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    acc[r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r], k) * uu.x);
                    acc[r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r + 1], k) * uu.y);
                    acc[r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r + 2], k) * uu.z);
                    acc[r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r + 3], k) * uu.w);
                }
            } else {
                // coefficients against B^T u (FP32); B is applied once to the
                // row group's sums below
                bool cut;
                decode_block_coeffs<NW, THREADS>(row, tab, w[0], emax, iv, cut);
                float ut[4];
                lin_bt_u<float>(uu.x, uu.y, uu.z, uu.w, ut);
                const int k = emax - 30;
                float v[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v[r] = (float)(int32_t)iv[4 * r] * ut[0];
                    v[r] = __builtin_fmaf((float)(int32_t)iv[4 * r + 1], ut[1], v[r]);
                    v[r] = __builtin_fmaf((float)(int32_t)iv[4 * r + 2], ut[2], v[r]);
                    v[r] = __builtin_fmaf((float)(int32_t)iv[4 * r + 3], ut[3], v[r]);
                }
                if (__any(cut) && cut) // rare: the exact lift, back to coefficient space
                    exact_block_sums(iv, uu, v);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[r].add(__builtin_ldexpf(v[r], k));
            }
        }
        // reduce the row's sums across the group's lanes within the wave
#pragma unroll
        for (int r = 0; r < 4; ++r)
            for (int mask = first_mask; mask >= 1; mask >>= 1)
                acc[r].merge_from_lane(mask);
        if constexpr (kShared)
            __syncthreads(); // every wave is done with its staging rows
        if (leader && bi < bi_end) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                red[slot * slot_len + 4 * t + r] = acc[r].value();
        }
        if constexpr (kShared)
            break; // one tile row (checked at launch)
    }

    // then across the waves of a group, one lane per block row (per row of
    // the matrix for the Fig. 7 sums)
    __syncthreads();
    const uint32_t nslots = wide ? G >> 6 : 1u;
    const uint32_t i = Acc::kPerProduct ? threadIdx.x >> 2 : threadIdx.x;
    const uint32_t g = i % groups, t = i / groups, bi = bi0 + t * groups + g;
    if (t >= rpg || bi >= bi_end)
        return;
    const uint32_t s0 = wide ? g * nslots : g;
    auto emit = [&](uint32_t r, double v) {
        const uint32_t local = (bi - bi_begin) * 4 + r;
        if (nslab > 1)
            part[(uint64_t)slab * ((bi_end - bi_begin) * 4) + local] = v;
        else if (local >= skip && local - skip < nrows)
            y[local - skip] = (float)v;
    };
    if constexpr (Acc::kPerProduct) {
        const uint32_t r = threadIdx.x & 3u;
        double v = red[s0 * slot_len + 4 * t + r];
        for (uint32_t q = 1; q < nslots; ++q)
            v += red[(s0 + q) * slot_len + 4 * t + r];
        emit(r, v);
    } else {
        double v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            v[r] = red[s0 * slot_len + 4 * t + r];
            for (uint32_t q = 1; q < nslots; ++q)
                v[r] += red[(s0 + q) * slot_len + 4 * t + r];
        }
        lin_inv_lift<double>(v[0], v[1], v[2], v[3]);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            emit((uint32_t)r, v[r]);
    }
}

// ---------------------------------------------------- multi-RHS (MFMA path)
// Y = M U^T for k right-hand sides (the paper's GEMV, Sec. 4.4, takes one
// vector; several at once is this library's addition).  A block's rows
// against U are B (C (B^T U)) (C its coefficients, B the inverse transform's
// linear part; see lin_inv_lift), so the matrix cores contract coefficients,
// not decoded values, against B^T U, and B is applied once to each block
// row's sums at the end.
//
// B^T U is computed once per call by a small kernel into a workspace laid out
// as the MFMA B operands (below); every wave then loads the operands of its
// block columns itself, so the main kernel has no workgroup barrier after its
// start: each wave runs on its own.
//
// Workgroup = mrhs_waves(NT) waves, a tile of 4 block rows per wave x a slab
// of block columns: 16 waves (1024 lanes) for up to 16 right-hand sides, so
// that two workgroups fit a CU in LDS and 32 waves in 64 VGPRs each; 8 waves
// for more, whose FP64 sums leave registers for 16 waves.  Per step of 16
// block columns, each lane decodes one block of its wave's 4 x 16 tile (with
// 8-wave workgroups the next step's block words are already in flight) and
// keeps its coefficients, scaled by the block's 2^(emax - 30), in registers;
// then
//   FP32 U   four quarters of 4 block columns: the quarter's lanes write their
//            blocks to the wave's 16 x 16 LDS tile, which is contracted with
//            v_mfma_f32_16x16x4f32, K = the quarter's 4 block columns, one
//            MFMA per coefficient column: 4 MFMAs per quarter and 16
//            right-hand sides
//   FP32 U,  up to 4 right-hand sides: the same quarters on
//   k <= 4   v_mfma_f32_4x4x1f32 (16 blocks of 4 x 4, K = 1; below,
//            mrhs_load_bn): 4 MFMAs per quarter, a quarter of the 16x16x4
//            cycles, which at k <= 4 would contract zero columns
//   BF16 U   two halves of 8 block columns, written rounded to BF16 and
//            contracted with v_mfma_f32_16x16x32_bf16 (K = 32), 1 MFMA per
//            half and 16 right-hand sides
//   X6       FP32 U from 17 right-hand sides up: the halves of the BF16
//            path, with every FP32 coefficient and every FP32 value of B^T U
//            split into three BF16 parts by truncation (x = x1 + x2 + x3
//            exactly: 8 significant bits each).  Of the nine products of
//            parts, the six whose order is at most 2^-16 of the whole (1.1,
//            1.2, 2.1, 1.3, 2.2, 3.1) are accumulated: 6 MFMAs per half and
//            16 right-hand sides.  Every BF16 product is exact in FP32, and
//            the three dropped ones are below 2^-21 of the product (the
//            split of Henry, Tang and Heinecke, "Leveraging the bfloat16
//            artificial intelligence datatype for higher-precision
//            computations", ARITH 2019).  BF16 MFMAs run beside the
//            decoder's VALU work, where FP32 ones do not
// Operand layouts (16x16 output tile D[i][j], lane l):
//   A[i][kk]  lane = i + 16*(kk/g), element kk % g   (g = 1 FP32, 8 BF16)
//   B[kk][j]  lane = j + 16*(kk/g), element kk % g
//   D[i][j]   lane = j + 16*(i/4), register i % 4
// so each lane's four accumulators are the four coefficient rows of one
// block row.  The FP32 MFMA accumulators cover one step (K = 64); after
// every step they are added into FP64 sums.
static_assert(4 * mrhs_waves(1, MrhsMath::F32) <= (int)kMrhsMaxTileBlockRows &&
                  4 * mrhs_waves(4, MrhsMath::F32) <= (int)kMrhsMaxTileBlockRows &&
                  4 * mrhs_waves(2, MrhsMath::X6) <= (int)kMrhsMaxTileBlockRows,
              "block rows per multi-RHS workgroup");
constexpr int kMathF32 = (int)MrhsMath::F32, kMathBf16 = (int)MrhsMath::Bf16, kMathX6 = (int)MrhsMath::X6,
              kMathF32N = (int)MrhsMath::F32N;
constexpr int kATileStride = 16 + 4; // floats per LDS row of a wave's X6 part tile (40 BF16)
constexpr int kATile32Stride = 16;    // floats per LDS row of a wave's FP32 quarter tile (swizzled)
typedef float mf32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 mbf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// an X6 part tile of a wave: 16 rows of 32 BF16 coefficients (8 block
// columns) plus 8 of padding
constexpr int kATile16Stride = 40;
static_assert(16 * kATile16Stride * 2 <= 16 * kATileStride * 4, "an X6 part tile fits its LDS");
constexpr int kATileBf16Stride = 32; // BF16 per LDS row of a wave's BF16 half tile (swizzled)

__device__ __forceinline__ uint16_t to_bf16_rne(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// x = x1 + x2 + x3 exactly, each part a BF16 value (8 significant bits, cut
// by truncation), returned as FP32 bit patterns whose low halves are zero.
__device__ __forceinline__ void split3_bf16(float x, uint32_t& x1, uint32_t& x2, uint32_t& x3)
{
    x1 = __float_as_uint(x) & 0xFFFF0000u;
    const float r = x - __uint_as_float(x1); // exact: the low 16 bits of x's significand
    x2 = __float_as_uint(r) & 0xFFFF0000u;
    x3 = __float_as_uint(r - __uint_as_float(x2)); // exact, at most 8 significant bits
}

// Two BF16 values (the high halves of two FP32 bit patterns) in one word,
// the first in the low half.
__device__ __forceinline__ uint32_t pack_hi16(uint32_t lo_src, uint32_t hi_src)
{
    return (lo_src >> 16) | (hi_src & 0xFFFF0000u);
}

// Orders the LDS accesses of the lanes of one wave: writes before it are
// visible to reads after it in every lane of the wave, and no access moves
// across it.
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// B^T U for NT groups of 16 right-hand sides (zero past k and past the last
// column), over nbc16 block columns (a multiple of 16; zero past the
// matrix), in the layout the MFMA B operands are loaded in:
//   FP32  float[bc][n][16][4]:      for lane (j, kk) of a quarter's K = 4
//                                   MFMAs (kk: block column), the four values
//                                   m = 0..3 of right-hand side 16 n + j:
//                                   one 16-byte load per quarter
//   BF16  bf16[bc / 2][n][16][8]:   for lane (j, g) of a K = 32 MFMA, the
//                                   eight values (bc & 1, m) of block
//                                   columns 2p, 2p + 1: one 16-byte load
//   X6    bf16[bc / 2][n][3][16][8]: the BF16 layout for each of the three
//                                   parts of the FP32 values
// One thread per (right-hand side, block column), block columns fastest so
// that the loads of U are contiguous.
template <int MATH>
__global__ void __launch_bounds__(kThreads) mrhs_btu_kernel(const void* __restrict__ Uv, uint32_t ldu, uint32_t k,
                                                            uint32_t nt, uint32_t cols, uint32_t nbc16,
                                                            void* __restrict__ out)
{
    constexpr bool BF16U = MATH == kMathBf16;
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= (uint64_t)nbc16 * 16 * nt)
        return;
    const uint32_t bc = (uint32_t)(i % nbc16), rhs = (uint32_t)(i / nbc16);
    float u0 = 0.f, u1 = 0.f, u2 = 0.f, u3 = 0.f;
    const uint32_t j = 4 * bc;
    if (rhs < k && j < cols) {
        const uint32_t nv = cols - j < 4u ? cols - j : 4u;
        const uint64_t o = (uint64_t)rhs * ldu + j;
        if constexpr (BF16U) {
            const uint16_t* U = static_cast<const uint16_t*>(Uv) + o;
            u0 = bf16_to_float(U[0]);
            u1 = nv > 1 ? bf16_to_float(U[1]) : 0.f;
            u2 = nv > 2 ? bf16_to_float(U[2]) : 0.f;
            u3 = nv > 3 ? bf16_to_float(U[3]) : 0.f;
        } else {
            const float* U = static_cast<const float*>(Uv) + o;
            u0 = U[0];
            u1 = nv > 1 ? U[1] : 0.f;
            u2 = nv > 2 ? U[2] : 0.f;
            u3 = nv > 3 ? U[3] : 0.f;
        }
    }
    float ut[4];
    lin_bt_u<float>(u0, u1, u2, u3, ut);
    const uint32_t n = rhs >> 4, jj = rhs & 15u;
    if constexpr (BF16U) {
        uint16_t* o = static_cast<uint16_t*>(out) + ((((uint64_t)(bc >> 1) * nt + n) * 16 + jj) * 8 + (bc & 1u) * 4);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            o[m] = to_bf16_rne(ut[m]);
    } else if constexpr (MATH == kMathX6) {
        uint16_t* o = static_cast<uint16_t*>(out) + ((((uint64_t)(bc >> 1) * nt + n) * 3 * 16 + jj) * 8 + (bc & 1u) * 4);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uint32_t p1, p2, p3;
            split3_bf16(ut[m], p1, p2, p3);
            o[m] = (uint16_t)(p1 >> 16);
            o[16 * 8 + m] = (uint16_t)(p2 >> 16);
            o[2 * 16 * 8 + m] = (uint16_t)(p3 >> 16);
        }
    } else {
        float* o = static_cast<float*>(out) + (((uint64_t)bc * nt + n) * 16 + jj) * 4;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            o[m] = ut[m];
    }
}

// Loads of a lane's block words (no LDS yet): NW words at g.
template <int NW>
__device__ __forceinline__ void load_block_words(const uint32_t* __restrict__ g, uint32_t (&w)[NW])
{
    if constexpr (NW % 4 == 0) {
        const u32x4* g4 = reinterpret_cast<const u32x4*>(g);
#pragma unroll
        for (int k = 0; k < NW / 4; ++k) {
            const u32x4 v = __builtin_nontemporal_load(g4 + k);
            w[4 * k] = v.x;
            w[4 * k + 1] = v.y;
            w[4 * k + 2] = v.z;
            w[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k)
            w[k] = g[k];
    }
}

// FP32 U: the B operands of one quarter (4 block columns from bc) for this
// lane (j = lane % 16, block column bc + lane / 16): B^T U's four values
// m = 0..3 of right-hand side 16 n + j, one MFMA each.
template <int NT>
__device__ __forceinline__ void mrhs_load_bq(const float* __restrict__ btf, uint32_t bc, int lane, f32x4 (&b)[NT])
{
    const uint32_t kk = (uint32_t)lane >> 4, j = (uint32_t)lane & 15u;
#pragma unroll
    for (int n = 0; n < NT; ++n)
        b[n] = *reinterpret_cast<const f32x4*>(btf + (((uint64_t)(bc + kk) * NT + n) * 16 + j) * 4);
}

// Quarters of B operands loaded ahead (FP32 U), as many as the registers for
// six (one group of right-hand sides) or four waves per SIMD leave room for.
template <int NT>
constexpr int kMrhsAhead = NT == 1 ? 1 : (NT == 2 ? 2 : 1);

// FP32 U, up to 4 right-hand sides on v_mfma_f32_4x4x1f32 (16 blocks of
// 4 x 4, K = 1), where the 16x16x4 MFMA would spend three quarters of its
// cycles on zero columns.  MFMA block b = 4 t + s of lane l (t = l / 16,
// s = l / 4 % 4) sums block row t over its share s of the block columns:
// of each quarter q of a step, block column 4 q + s, one MFMA per
// coefficient column m; j = l % 4 is the right-hand side.  The B operands of
// quarter q of a step for this lane: B^T U's four values m = 0..3 for
// right-hand side j at block column cb + 4 q + s, from the FP32 layout of
// one group of 16.
__device__ __forceinline__ void mrhs_load_bn(const float* __restrict__ btf, uint32_t cb, int qi, int lane, f32x4& b)
{
    const uint32_t sh = ((uint32_t)lane >> 2) & 3u, j = (uint32_t)lane & 3u;
    const uint32_t bc = cb + 4u * (uint32_t)qi + sh;
    b = *reinterpret_cast<const f32x4*>(btf + ((uint64_t)bc * 16 + j) * 4);
}
constexpr int kMrhsNarrowAhead = 1;
static_assert(kMrhsNarrowMax <= 4, "the 4x4x1 path holds one group of 4 right-hand sides");
static_assert(16 * kATile32Stride >= 4 * 4 * 16, "a quarter's 16 blocks fit the FP32 tile");

// X6: the B operand words (three parts, 16 bytes each) of one half and one
// group of 16 right-hand sides for this lane.
template <int NT>
__device__ __forceinline__ void mrhs_load_bx(const uint16_t* __restrict__ btb, uint32_t cb, int h, int n, int lane,
                                             u32x4 (&b)[3])
{
    const uint32_t g = (uint32_t)lane >> 4, j = (uint32_t)lane & 15u;
    const uint16_t* p = btb + ((((uint64_t)(cb / 2 + 4 * h + g) * NT + n) * 3 * 16 + j) * 8);
#pragma unroll
    for (int q = 0; q < 3; ++q)
        b[q] = *reinterpret_cast<const u32x4*>(p + q * 16 * 8);
}

// X6: (half, group) B parts loaded ahead of their MFMAs, the first of them
// before the decode (one, two or three ahead time the same at 65536^2, k = 64:
// 7.29 / 7.27 / 7.28 ms; two take the fewest registers).
constexpr int kX6Ahead = 2;

// two workgroups per CU, i.e. W / 2 waves per SIMD: the register budget the
// compiler must meet (64 VGPRs at 16 waves, 128 at 8)
template <int NW, int MATH, int NT>
__global__ void __launch_bounds__(64 * mrhs_waves(NT, (MrhsMath)MATH), mrhs_waves(NT, (MrhsMath)MATH) / 2)
    mrhs_kernel(const uint32_t* __restrict__ stream, const void* __restrict__ btu, uint32_t k, float* __restrict__ Y,
                uint32_t ldy, double* __restrict__ part, uint32_t nbc, uint32_t bi_begin, uint32_t bi_end,
                uint32_t slab_bc, uint32_t nslab, uint32_t nrows_out)
{
    constexpr bool BF16U = MATH == kMathBf16, X6 = MATH == kMathX6, NARROW = MATH == kMathF32N;
    constexpr int W = mrhs_waves(NT, (MrhsMath)MATH), T = 64 * W;
    // accumulator tiles per lane: one per group of 16 right-hand sides, or
    // one for the 4x4x1 path (its groups of 4 lie in different lanes)
    constexpr int NA = NARROW ? 1 : NT;
    __shared__ uint32_t lds[T * kStagedWords<NW>];
    __shared__ uint32_t tab[kSecEntries];
    // the wave's A tile: FP32 quarters (16 x 16, swizzled), BF16 halves
    // (16 x 32, swizzled), or three BF16 halves (one per part) for X6
    __shared__ __align__(16) float atile[W][X6 ? 3 * 16 * kATileStride
                                              : (BF16U ? 16 * kATileBf16Stride / 2 : 16 * kATile32Stride)];
    uint32_t* row = lds + threadIdx.x;
    clear_pad<NW, T>(row);
    load_section_table<T>(tab); // the last workgroup barrier

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t bw = bi_begin + tile * (4 * W) + 4 * wave; // first block-row of this wave
    const uint32_t bc0 = slab * slab_bc;
    const uint32_t bc1 = bc0 + slab_bc < nbc ? bc0 + slab_bc : nbc;
    const int t = lane >> 4, c = lane & 15; // this lane's block in the wave's 4 x 16 step tile
    const uint32_t bi = bw + t;
    float* at = atile[wave];
    const float* btf = static_cast<const float*>(btu);
    const uint16_t* btb = static_cast<const uint16_t*>(btu);

    // 16-wave workgroups load each step's block words at the step (their
    // registers hold no next step's words); smaller ones keep them in flight
    // one step ahead
    constexpr bool kAhead = W < 16;
    uint32_t w[NW];
    if constexpr (kAhead) {
        const bool valid = bi < bi_end && bc0 + c < bc1;
        if (valid)
            load_block_words<NW>(stream + ((uint64_t)bi * nbc + bc0 + c) * NW, w);
        else
#pragma unroll
            for (int q = 0; q < NW; ++q)
                w[q] = 0u; // decodes as a zero block
    }

    mf32x4 acc[NA];
    double sum[NA][4];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            sum[n][j] = 0.0;

    for (uint32_t cb = bc0; cb < bc1; cb += 16) {
        // ---- this step's block words to the lane's LDS row; the next
        // step's in flight
        if constexpr (!kAhead) {
            const bool valid = bi < bi_end && cb + c < bc1;
            if (valid)
                load_block_words<NW>(stream + ((uint64_t)bi * nbc + cb + c) * NW, w);
            else
#pragma unroll
                for (int q = 0; q < NW; ++q)
                    w[q] = 0u;
        }
#pragma unroll
        for (int q = 0; q < NW; ++q)
            row[q * T] = w[q];
        const uint32_t w0 = w[0];
        if constexpr (kAhead) {
            const bool valid = bi < bi_end && cb + 16 + c < bc1;
            if (valid)
                load_block_words<NW>(stream + ((uint64_t)bi * nbc + cb + 16 + c) * NW, w);
            else
#pragma unroll
                for (int q = 0; q < NW; ++q)
                    w[q] = 0u;
        }
        // ---- B operands in flight during the decode (block columns cb ..
        // cb + 15 lie inside the workspace: it spans whole steps)
        constexpr int AH = NARROW ? kMrhsNarrowAhead : kMrhsAhead<NT>;
        f32x4 bq[MATH == kMathF32 || NARROW ? AH : 1][NARROW ? 1 : NT];
        u32x4 bh[BF16U ? 2 : 1][NT];
        // X6: the B parts of the (half, group) in use and the kX6Ahead after it
        u32x4 bx[X6 ? kX6Ahead + 1 : 1][3];
        if constexpr (X6) {
#pragma unroll
            for (int i = 0; i < kX6Ahead; ++i)
                mrhs_load_bx<NT>(btb, cb, i / NT, i % NT, lane, bx[i]);
        } else if constexpr (BF16U) {
            // the second half's operands load once the first half starts
            // when 16 waves share the registers
            const uint32_t g = (uint32_t)lane >> 4, j = (uint32_t)lane & 15u;
#pragma unroll
            for (int h = 0; h < (W >= 16 ? 1 : 2); ++h)
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    bh[h][n] = *reinterpret_cast<const u32x4*>(
                        btb + (((uint64_t)(cb / 2 + 4 * h + g) * NT + n) * 16 + j) * 8);
        } else if constexpr (NARROW) {
#pragma unroll
            for (int q = 0; q < AH; ++q)
                mrhs_load_bn(btf, cb, q, lane, bq[q][0]);
        } else {
#pragma unroll
            for (int q = 0; q < AH; ++q)
                mrhs_load_bq<NT>(btf, cb + 4 * q, lane, bq[q]);
        }
        // ---- decode one block per lane: scaled coefficients (registers)
        int emax;
        uint32_t cf[16];
        bool cut;
        decode_block_coeffs<NW, T>(row, tab, w0, emax, cf, cut);
        float sc[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
            sc[v] = __builtin_ldexpf((float)(int32_t)cf[v], emax - 30);
        if (__any(cut) && cut) // rare: the exact lift (see exact_block_coeffs)
            exact_block_coeffs(cf, emax, sc);
#pragma unroll
        for (int n = 0; n < NA; ++n)
            acc[n] = mf32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (NARROW) {
            // ---- four quarters of 4 block columns (the MFMA blocks and
            // shares of mrhs_load_bn): the quarter's lanes write their blocks
            // to the wave's tile as [t][s][r][m], then lane (t, s, r) reads
            // row r of its share's block column and runs its 4 MFMAs (A: lane
            // r + 4 b holds A_b[r]; B: lane j + 4 b holds B_b[j]; D_b[r][j]:
            // lane j + 4 b, register r)
            const int tn = lane >> 4, sn = (lane >> 2) & 3, rn = lane & 3;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                wave_sync_lds();
                if ((c >> 2) == q) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        *reinterpret_cast<f32x4*>(at + ((t * 4 + (c & 3)) * 4 + r) * 4) =
                            f32x4{sc[4 * r], sc[4 * r + 1], sc[4 * r + 2], sc[4 * r + 3]};
                }
                wave_sync_lds();
                const int slot = q % AH;
                const f32x4 a4 = *reinterpret_cast<const f32x4*>(at + ((tn * 4 + sn) * 4 + rn) * 4);
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    acc[0] = __builtin_amdgcn_mfma_f32_4x4x1f32(a4[m], bq[slot][0][m], acc[0], 0, 0, 0);
                if (q + AH < 4) // the quarter AH on into the slot just used
                    mrhs_load_bn(btf, cb, q + AH, lane, bq[slot][0]);
            }
        } else if constexpr (MATH == kMathF32) {
            // ---- four quarters of 4 block columns: the quarter's lanes write
            // their blocks to the wave's 16 x 16 tile (row 4t + r, a 4-float
            // group per block column, the group index XORed with t so that
            // the column reads below spread over the banks), then every lane
            // reads its A operands
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // the tile is the wave's own: lanes read what other lanes of
                // the wave wrote, so each hand-over is a wave-scope
                // release/acquire (no workgroup barrier is needed)
                wave_sync_lds();
                if ((c >> 2) == q) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        *reinterpret_cast<f32x4*>(at + (4 * t + r) * kATile32Stride + 4 * ((c & 3) ^ t)) =
                            f32x4{sc[4 * r], sc[4 * r + 1], sc[4 * r + 2], sc[4 * r + 3]};
                }
                wave_sync_lds();
                const int slot = q % AH, ar = lane & 15;
                // MFMA m contracts coefficient column m of the quarter's four
                // block columns (K = block column): lane l holds A[l % 16][l / 16],
                // coefficient (r, m) = ((l % 16) % 4, m) of block column l / 16
                const f32x4 a4 =
                    *reinterpret_cast<const f32x4*>(at + ar * kATile32Stride + 4 * ((lane >> 4) ^ (ar >> 2)));
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[m], bq[slot][n][m], acc[n], 0, 0, 0);
                if (q + AH < 4) // the quarter after next into the slot just used
                    mrhs_load_bq<NT>(btf, cb + 4 * (q + AH), lane, bq[slot]);
            }
        } else if constexpr (X6) {
            // ---- the coefficients' three BF16 parts, packed in pairs; both
            // halves' A operands are read before any MFMA, so that the packed
            // words die first (the tile is then written twice)
            uint32_t pk[3][8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                uint32_t a1, a2, a3, b1, b2, b3;
                split3_bf16(sc[2 * v], a1, a2, a3);
                split3_bf16(sc[2 * v + 1], b1, b2, b3);
                pk[0][v] = pack_hi16(a1, b1);
                pk[1][v] = pack_hi16(a2, b2);
                pk[2][v] = pack_hi16(a3, b3);
            }
            uint16_t* at16 = reinterpret_cast<uint16_t*>(at);
            constexpr int kPart = 16 * kATile16Stride; // BF16 elements per part's tile
            u32x4 av[2][3];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                wave_sync_lds();
                if ((c >> 3) == h) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            *reinterpret_cast<u32x2*>(at16 + q * kPart + (4 * t + r) * kATile16Stride + 4 * (c & 7)) =
                                u32x2{pk[q][2 * r], pk[q][2 * r + 1]};
                }
                wave_sync_lds();
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    av[h][q] = *reinterpret_cast<const u32x4*>(at16 + q * kPart + (lane & 15) * kATile16Stride +
                                                               8 * (lane >> 4));
            }
            // ---- per half and group of 16 right-hand sides, six MFMAs; the
            // B parts of the next (half, group) load meanwhile
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const int i = h * NT + n, cur = i % (kX6Ahead + 1);
                    if (i + kX6Ahead < 2 * NT)
                        mrhs_load_bx<NT>(btb, cb, (i + kX6Ahead) / NT, (i + kX6Ahead) % NT, lane,
                                         bx[(i + kX6Ahead) % (kX6Ahead + 1)]);
                    const mbf16x8 a1 = __builtin_bit_cast(mbf16x8, av[h][0]);
                    const mbf16x8 a2 = __builtin_bit_cast(mbf16x8, av[h][1]);
                    const mbf16x8 a3 = __builtin_bit_cast(mbf16x8, av[h][2]);
                    const mbf16x8 b1 = __builtin_bit_cast(mbf16x8, bx[cur][0]);
                    const mbf16x8 b2 = __builtin_bit_cast(mbf16x8, bx[cur][1]);
                    const mbf16x8 b3 = __builtin_bit_cast(mbf16x8, bx[cur][2]);
                    // smallest products first
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b1, acc[n], 0, 0, 0);
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2, acc[n], 0, 0, 0);
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b3, acc[n], 0, 0, 0);
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b1, acc[n], 0, 0, 0);
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b2, acc[n], 0, 0, 0);
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[n], 0, 0, 0);
                }
        } else {
            // ---- two halves of 8 block columns (K = 32): the lanes of a half
            // write their blocks' coefficients, rounded to BF16, to the 16 x
            // 32 tile (row 4t + r, columns 4 (c % 8) .. + 3, each 16-byte
            // pair of block columns XORed with t so that the reads below
            // spread over the banks); lane l then holds A[l % 16][8 (l / 16)
            // .. + 7] (two block columns) and B[8 (l / 16) .. + 7][l % 16]
            uint16_t* at16 = reinterpret_cast<uint16_t*>(at);
            uint32_t pk[8];
#pragma unroll
            for (int v = 0; v < 8; ++v)
                pk[v] = (uint32_t)to_bf16_rne(sc[2 * v]) | (uint32_t)to_bf16_rne(sc[2 * v + 1]) << 16;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (W >= 16 && h == 1) {
                    const uint32_t g = (uint32_t)lane >> 4, j = (uint32_t)lane & 15u;
#pragma unroll
                    for (int n = 0; n < NT; ++n)
                        bh[1][n] = *reinterpret_cast<const u32x4*>(
                            btb + (((uint64_t)(cb / 2 + 4 + g) * NT + n) * 16 + j) * 8);
                }
                wave_sync_lds();
                if ((c >> 3) == h) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        *reinterpret_cast<u32x2*>(at16 + (4 * t + r) * kATileBf16Stride +
                                                  8 * (((c & 7) >> 1) ^ t) + 4 * (c & 1)) = u32x2{pk[2 * r], pk[2 * r + 1]};
                }
                wave_sync_lds();
                const int ar = lane & 15;
                const u32x4 av = *reinterpret_cast<const u32x4*>(at16 + ar * kATileBf16Stride +
                                                                 8 * ((lane >> 4) ^ (ar >> 2)));
                const mbf16x8 a = __builtin_bit_cast(mbf16x8, av);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(mbf16x8, bh[h][n]), acc[n],
                                                                     0, 0, 0);
            }
        }
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sum[n][j] += (double)acc[n][j];
    }

    // ---- 4x4x1 sums: lane (t, s, j) holds block row t's sums over its
    // share s of the block columns for right-hand side j; the four shares
    // are added (the same order in every lane).  lane % 16 = j + 4 s: the
    // share-0 lanes hold their right-hand sides as in the 16x16 layout, the
    // others land on right-hand sides >= 4 >= k
    if constexpr (NARROW) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sum[0][j] += __shfl_xor(sum[0][j], 4, 64);
            sum[0][j] += __shfl_xor(sum[0][j], 8, 64);
        }
    }
    // ---- B on each block row's four coefficient-row sums; D[i][j]: lane
    // holds rows 4*(lane/16) + j, right-hand side lane%16
    const uint32_t nrows = (bi_end - bi_begin) * 4;
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        lin_inv_lift<double>(sum[n][0], sum[n][1], sum[n][2], sum[n][3]);
        const uint32_t rhs = 16 * n + (lane & 15);
        if (rhs >= k)
            continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t r = (bw - bi_begin) * 4 + 4 * (lane >> 4) + j;
            if (r >= nrows)
                continue;
            if (nslab > 1)
                part[((uint64_t)slab * k + rhs) * nrows + r] = sum[n][j];
            else if (r < nrows_out)
                Y[(uint64_t)rhs * ldy + r] = (float)sum[n][j];
        }
    }
}

// Slab partials [nslab][k][part_rows] -> Y (k x nrows, leading dimension
// ldy; nrows <= part_rows: the block-rows' padding is not written).
__global__ void __launch_bounds__(kThreads) reduce_slabs_batched_kernel(const double* __restrict__ part,
                                                                        uint32_t part_rows, uint32_t nrows,
                                                                        uint32_t k, uint32_t nslab,
                                                                        float* __restrict__ Y, uint32_t ldy)
{
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= (uint64_t)nrows * k)
        return;
    const uint32_t rhs = (uint32_t)(i / nrows), r = (uint32_t)(i % nrows);
    double s = 0.0;
    for (uint32_t q = 0; q < nslab; ++q)
        s += part[((uint64_t)q * k + rhs) * part_rows + r];
    Y[(uint64_t)rhs * ldy + r] = (float)s;
}

// Slab partials [nslab][part_rows] -> y[0, nrows), y[i] from partial row
// skip + i.  A wave takes 64 / L consecutive rows; the L lanes of a row sum
// a stride of its slabs each (a load reads 64 / L consecutive rows of L
// slabs), then add their sums in a fixed tree (the same order on every run).
template <int L>
__global__ void __launch_bounds__(kThreads) reduce_slabs_kernel(const double* __restrict__ part, uint32_t part_rows,
                                                                uint32_t skip, uint32_t nrows, uint32_t nslab,
                                                                float* __restrict__ y)
{
    constexpr uint32_t R = 64 / L;
    const uint32_t lane = threadIdx.x & 63, rr = lane % R, phase = lane / R;
    const uint64_t nwaves = ((uint64_t)nrows + R - 1) / R;
    const uint64_t wstride = (uint64_t)gridDim.x * (kThreads / 64);
    for (uint64_t w = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) / 64; w < nwaves; w += wstride) {
        const uint64_t i = w * R + rr;
        double s = 0.0;
        if (i < nrows)
            for (uint32_t q = phase; q < nslab; q += L)
                s += part[(uint64_t)q * part_rows + skip + i];
#pragma unroll
        for (uint32_t mask = 32; mask >= R; mask >>= 1)
            s += __shfl_xor(s, (int)mask, 64);
        if (i < nrows && phase == 0)
            y[i] = (float)s;
    }
}

unsigned grid_for(uint64_t items, unsigned cap = 1u << 20)
{
    uint64_t g = (items + kThreads - 1) / kThreads;
    if (g == 0)
        g = 1;
    return (unsigned)(g < cap ? g : cap);
}

template <int NW>
hipError_t launch_decode_blocks(const uint32_t* s, uint64_t b0, uint64_t n, float* out, hipStream_t st)
{
    hipLaunchKernelGGL(decode_blocks_kernel<NW>, dim3(grid_for(n, 65536)), dim3(kThreads), 0, st, s, b0, n, out);
    return hipGetLastError();
}

template <int NW>
hipError_t launch_decode_matrix(const uint32_t* s, uint32_t rows, uint32_t cols, float* out, hipStream_t st)
{
    const uint32_t nbr = (uint32_t)(((uint64_t)rows + 3) / 4), nbc = (uint32_t)(((uint64_t)cols + 3) / 4);
    const uint32_t npc = (nbc + 7) / 8;
    const uint64_t npatch = (uint64_t)((nbr + 7) / 8) * npc;
    constexpr uint64_t waves = kDecThreads<NW> / 64;
    const uint64_t g = (npatch + waves - 1) / waves;
    hipLaunchKernelGGL(decode_matrix_kernel<NW>, dim3((unsigned)(g == 0 ? 1 : (g < 65536 ? g : 65536))),
                       dim3(kDecThreads<NW>), 0, st, s, nbr, nbc, npc, npatch, rows, cols, out);
    return hipGetLastError();
}

template <int NW>
hipError_t launch_encode(const float* M, uint32_t rows, uint32_t cols, uint32_t* s, uint32_t* bad, hipStream_t st)
{
    const uint32_t nbc = (cols + 3) / 4;
    const uint64_t nb = (uint64_t)((rows + 3) / 4) * nbc;
    hipLaunchKernelGGL(encode_kernel<NW>, dim3(grid_for(nb, 65536)), dim3(kThreads), 0, st, M, nbc, rows, cols, nb, s,
                       bad);
    return hipGetLastError();
}

template <int NW, typename Acc>
hipError_t launch_gemv_t(const GemvPlan& pl, const uint32_t* s, const float* u, float* y, double* part,
                         hipStream_t st)
{
    if (pl.lanes != (uint32_t)kGemvThreads<NW>) // a plan made for another rate
        return hipErrorInvalidValue;
    if (kGemvSumsInStaging<NW> && pl.rpg != 1) // the row sums over the staging rows hold one tile row
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemv_kernel<NW, Acc>), dim3(pl.ntiles * pl.nslab), dim3(kGemvThreads<NW>), 0, st, s, u, y,
                       part, pl.nbc, pl.bi_begin, pl.bi_end, pl.slab_bc, pl.nslab, pl.cols, pl.nrows, pl.lg, pl.rpg,
                       pl.skip);
    return hipGetLastError();
}

template <int NW>
hipError_t launch_gemv(const GemvPlan& pl, AccMode mode, const uint32_t* s, const float* u, float* y, double* part,
                       hipStream_t st)
{
    hipError_t e = mode == AccMode::TwoSum  ? launch_gemv_t<NW, TwoSumAcc>(pl, s, u, y, part, st)
                   : mode == AccMode::PaperMp ? launch_gemv_t<NW, PaperMpAcc>(pl, s, u, y, part, st)
                                              : launch_gemv_t<NW, Fp64Acc>(pl, s, u, y, part, st);
    if (e != hipSuccess || pl.nslab == 1)
        return e;
    const uint32_t pr = pl.part_rows();
    if (pl.nslab <= 4)
        hipLaunchKernelGGL(reduce_slabs_kernel<1>, dim3(grid_for(pl.nrows)), dim3(kThreads), 0, st, part, pr, pl.skip,
                           pl.nrows, pl.nslab, y);
    else if (pl.nslab <= 64)
        hipLaunchKernelGGL(reduce_slabs_kernel<8>, dim3(grid_for((uint64_t)pl.nrows * 8)), dim3(kThreads), 0, st,
                           part, pr, pl.skip, pl.nrows, pl.nslab, y);
    else
        hipLaunchKernelGGL(reduce_slabs_kernel<64>, dim3(grid_for((uint64_t)pl.nrows * 64)), dim3(kThreads), 0, st,
                           part, pr, pl.skip, pl.nrows, pl.nslab, y);
    return hipGetLastError();
}

template <int NW, int MATH, int NT>
hipError_t launch_mrhs_t(const MrhsPlan& pl, const uint32_t* s, const void* btu, uint32_t k, float* Y, uint32_t ldy,
                         double* part, hipStream_t st)
{
    hipLaunchKernelGGL((mrhs_kernel<NW, MATH, NT>), dim3(pl.ntiles * pl.nslab),
                       dim3(64 * mrhs_waves(NT, (MrhsMath)MATH)), 0, st, s, btu, k, Y, ldy, part, pl.nbc, pl.bi_begin,
                       pl.bi_end, pl.slab_bc, pl.nslab, pl.nrows);
    return hipGetLastError();
}

template <int NW>
hipError_t launch_mrhs(const MrhsPlan& pl, const uint32_t* s, const void* U, uint32_t ldu, uint32_t k, float* Y,
                       uint32_t ldy, double* ws, hipStream_t st)
{
    const int nt = (int)((k + 15) / 16);
    const MrhsMath math = (MrhsMath)pl.math;
    if (math == MrhsMath::X6 && nt < 2)
        return hipErrorInvalidValue; // the planner gives X6 only from 17 right-hand sides up
    const MrhsWorkspace w = mrhs_workspace(pl, k);
    double* part = pl.nslab > 1 ? ws : nullptr;
    void* btu = ws + w.btu_offset;
    const uint32_t nbc16 = (pl.nbc + 15) / 16 * 16;
    const uint64_t items = (uint64_t)nbc16 * 16 * nt;
    const dim3 bgrid((unsigned)((items + kThreads - 1) / kThreads));
    if (math == MrhsMath::Bf16)
        hipLaunchKernelGGL(mrhs_btu_kernel<kMathBf16>, bgrid, dim3(kThreads), 0, st, U, ldu, k, (uint32_t)nt, pl.cols,
                           nbc16, btu);
    else if (math == MrhsMath::X6)
        hipLaunchKernelGGL(mrhs_btu_kernel<kMathX6>, bgrid, dim3(kThreads), 0, st, U, ldu, k, (uint32_t)nt, pl.cols,
                           nbc16, btu);
    else
        hipLaunchKernelGGL(mrhs_btu_kernel<kMathF32>, bgrid, dim3(kThreads), 0, st, U, ldu, k, (uint32_t)nt, pl.cols,
                           nbc16, btu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (math == MrhsMath::F32N) {
        if (k > kMrhsNarrowMax)
            return hipErrorInvalidValue; // the planner gives the 4x4x1 path only up to kMrhsNarrowMax
        e = launch_mrhs_t<NW, kMathF32N, 1>(pl, s, btu, k, Y, ldy, part, st);
    } else switch (nt * 3 + (int)math) {
    case 3: e = launch_mrhs_t<NW, kMathF32, 1>(pl, s, btu, k, Y, ldy, part, st); break;
    case 4: e = launch_mrhs_t<NW, kMathBf16, 1>(pl, s, btu, k, Y, ldy, part, st); break;
    case 6: e = launch_mrhs_t<NW, kMathF32, 2>(pl, s, btu, k, Y, ldy, part, st); break;
    case 7: e = launch_mrhs_t<NW, kMathBf16, 2>(pl, s, btu, k, Y, ldy, part, st); break;
    case 8: e = launch_mrhs_t<NW, kMathX6, 2>(pl, s, btu, k, Y, ldy, part, st); break;
    case 9: e = launch_mrhs_t<NW, kMathF32, 3>(pl, s, btu, k, Y, ldy, part, st); break;
    case 10: e = launch_mrhs_t<NW, kMathBf16, 3>(pl, s, btu, k, Y, ldy, part, st); break;
    case 11: e = launch_mrhs_t<NW, kMathX6, 3>(pl, s, btu, k, Y, ldy, part, st); break;
    case 12: e = launch_mrhs_t<NW, kMathF32, 4>(pl, s, btu, k, Y, ldy, part, st); break;
    case 13: e = launch_mrhs_t<NW, kMathBf16, 4>(pl, s, btu, k, Y, ldy, part, st); break;
    case 14: e = launch_mrhs_t<NW, kMathX6, 4>(pl, s, btu, k, Y, ldy, part, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || pl.nslab == 1)
        return e;
    hipLaunchKernelGGL(reduce_slabs_batched_kernel, dim3(grid_for((uint64_t)pl.nrows * k)), dim3(kThreads), 0, st,
                       part, pl.part_rows(), pl.nrows, k, pl.nslab, Y, ldy);
    return hipGetLastError();
}

} // namespace

} // namespace wh

// ---------------------------------------------------------------- exports
// This file is compiled once per words-per-block value WH_NW (rate = 2*WH_NW).
#ifndef WH_NW
#error "compile with -DWH_NW=<words per block>"
#endif
#define WH_CAT_(a, b) a##b
#define WH_CAT(a, b) WH_CAT_(a, b)

namespace wh {
namespace WH_CAT(nw, WH_NW) {

hipError_t decode_blocks(const void* stream, uint64_t b0, uint64_t n, float* out, hipStream_t st)
{
    return launch_decode_blocks<WH_NW>(static_cast<const uint32_t*>(stream), b0, n, out, st);
}

hipError_t decode_matrix(const void* stream, uint32_t rows, uint32_t cols, float* out, hipStream_t st)
{
    return launch_decode_matrix<WH_NW>(static_cast<const uint32_t*>(stream), rows, cols, out, st);
}

hipError_t encode(const float* M, uint32_t rows, uint32_t cols, void* stream, uint32_t* bad, hipStream_t st)
{
    return launch_encode<WH_NW>(M, rows, cols, static_cast<uint32_t*>(stream), bad, st);
}

hipError_t gemv(const GemvPlan& pl, AccMode mode, const void* stream, const float* u, float* y, double* part,
                hipStream_t st)
{
    return launch_gemv<WH_NW>(pl, mode, static_cast<const uint32_t*>(stream), u, y, part, st);
}

hipError_t mrhs(const MrhsPlan& pl, const void* stream, const void* U, uint32_t ldu, uint32_t k, float* Y,
                uint32_t ldy, double* part, hipStream_t st)
{
    return launch_mrhs<WH_NW>(pl, static_cast<const uint32_t*>(stream), U, ldu, k, Y, ldy, part, st);
}

} // namespace nwN
} // namespace wh
