// whz_kernels.hip -- WHZ1 kernels for gfx950: decode probe, full decode,
// encoder, and the fused decode + mixed-precision GEMV (k = 1).
//
// Fused GEMV (the deformation product y = C.S of Eq. 2 over a zfp-compressed
// matrix, Sec. 4.3-4.4):
//   grid     one workgroup (256 lanes, 4 waves) per (row tile, column slab);
//            a row tile is TR block-rows (4*TR rows)
//   lane     decodes one 4x4 block per step: the 256 lanes of a workgroup
//            take 256 consecutive blocks of a block-row, so every step reads
//            one contiguous run of the stream (16*rate*256/8 bytes)
//   u        the lane's 4 values of u are loaded once per step and reused
//            for all TR block-rows of the tile
//   sums     FP32 within a block row (4 products), then FP64 (or
//            compensated FP32) across blocks; wave shuffles + LDS for the
//            reduction across lanes; one FP64 partial per row and slab
//   reduce   a second kernel adds the slab partials in FP64 and rounds once
//            to FP32 (skipped when there is a single slab)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "whz_device.hpp"
#include "wh_internal.hpp"

namespace wh {
namespace {

constexpr int kThreads = 256;

template <int NW>
struct LdsRow {
    static constexpr int kStride = NW + 3; // odd for even NW: no bank conflicts
};

// Stage one block (NW words at g) into this lane's LDS row.
template <int NW>
__device__ __forceinline__ void stage_block(uint32_t* row, const uint32_t* __restrict__ g, uint32_t (&w)[NW])
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
        row[k] = w[k];
}

template <int NW>
__device__ __forceinline__ void clear_pad(uint32_t* row)
{
    row[NW] = 0u;
    row[NW + 1] = 0u;
    row[NW + 2] = 0u;
}

// ------------------------------------------------------- decode kernels
template <int NW>
__global__ void __launch_bounds__(kThreads) decode_blocks_kernel(const uint32_t* __restrict__ stream, uint64_t b0,
                                                                 uint64_t nblocks, float* __restrict__ out)
{
    __shared__ uint32_t lds[kThreads * LdsRow<NW>::kStride];
    uint32_t* row = lds + threadIdx.x * LdsRow<NW>::kStride;
    clear_pad<NW>(row);
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < nblocks; i += stride) {
        uint32_t w[NW];
        stage_block<NW>(row, stream + (b0 + i) * NW, w);
        int emax;
        uint32_t iv[16];
        decode_block_ints<NW>(row, w[0], emax, iv);
        float4* o = reinterpret_cast<float4*>(out + 16 * i);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            o[r] = make_float4(__builtin_ldexpf((float)(int32_t)iv[4 * r], emax - 30),
                               __builtin_ldexpf((float)(int32_t)iv[4 * r + 1], emax - 30),
                               __builtin_ldexpf((float)(int32_t)iv[4 * r + 2], emax - 30),
                               __builtin_ldexpf((float)(int32_t)iv[4 * r + 3], emax - 30));
    }
}

// Whole matrix into row-major FP32 (rows x cols).
template <int NW>
__global__ void __launch_bounds__(kThreads) decode_matrix_kernel(const uint32_t* __restrict__ stream, uint32_t nbc,
                                                                 uint64_t nblocks, uint32_t cols,
                                                                 float* __restrict__ out)
{
    __shared__ uint32_t lds[kThreads * LdsRow<NW>::kStride];
    uint32_t* row = lds + threadIdx.x * LdsRow<NW>::kStride;
    clear_pad<NW>(row);
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < nblocks; b += stride) {
        uint32_t w[NW];
        stage_block<NW>(row, stream + b * NW, w);
        int emax;
        uint32_t iv[16];
        decode_block_ints<NW>(row, w[0], emax, iv);
        const uint64_t bi = b / nbc, bj = b % nbc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            f32x4 v;
            v.x = __builtin_ldexpf((float)(int32_t)iv[4 * r], emax - 30);
            v.y = __builtin_ldexpf((float)(int32_t)iv[4 * r + 1], emax - 30);
            v.z = __builtin_ldexpf((float)(int32_t)iv[4 * r + 2], emax - 30);
            v.w = __builtin_ldexpf((float)(int32_t)iv[4 * r + 3], emax - 30);
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(out + (4 * bi + r) * cols + 4 * bj));
        }
    }
}

// ---------------------------------------------------------------- encoder
template <int NW>
__global__ void __launch_bounds__(kThreads) encode_kernel(const float* __restrict__ M, uint32_t nbc, uint32_t cols,
                                                          uint64_t nblocks, uint32_t* __restrict__ stream,
                                                          uint32_t* __restrict__ bad)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < nblocks; b += stride) {
        const uint64_t bi = b / nbc, bj = b % nbc;
        float f[16];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float4 v = *reinterpret_cast<const float4*>(M + (4 * bi + r) * cols + 4 * bj);
            f[4 * r] = v.x;
            f[4 * r + 1] = v.y;
            f[4 * r + 2] = v.z;
            f[4 * r + 3] = v.w;
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

template <int NW, int TR, typename Acc>
__global__ void __launch_bounds__(kThreads) gemv_kernel(const uint32_t* __restrict__ stream,
                                                        const float* __restrict__ u, float* __restrict__ y,
                                                        double* __restrict__ part, uint32_t nbc, uint32_t bi_begin,
                                                        uint32_t bi_end, uint32_t slab_bc, uint32_t nslab)
{
    __shared__ uint32_t lds[kThreads * LdsRow<NW>::kStride];
    __shared__ double red[kThreads / 64][TR * 4];
    uint32_t* row = lds + threadIdx.x * LdsRow<NW>::kStride;
    clear_pad<NW>(row);

    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t bi0 = bi_begin + tile * TR;
    const uint32_t nr = bi_end - bi0 < (uint32_t)TR ? bi_end - bi0 : (uint32_t)TR;
    const uint32_t bc0 = slab * slab_bc;
    const uint32_t bc1 = bc0 + slab_bc < nbc ? bc0 + slab_bc : nbc;

    Acc acc[TR][4];
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[t][r].zero();

    for (uint32_t bj = bc0 + threadIdx.x; bj < bc1; bj += kThreads) {
        const float4 uu = reinterpret_cast<const float4*>(u)[bj];
#pragma unroll
        for (int t = 0; t < TR; ++t) {
            if ((uint32_t)t < nr) {
                uint32_t w[NW];
                stage_block<NW>(row, stream + ((uint64_t)(bi0 + t) * nbc + bj) * NW, w);
                int emax;
                uint32_t iv[16];
                decode_block_ints<NW>(row, w[0], emax, iv);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if constexpr (Acc::kPerProduct) {
                        // Fig. 7: each FP32 product of the decoded value and
                        // u is added to the FP64 sum on its own
                        const int k = emax - 30;
                        acc[t][r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r], k) * uu.x);
                        acc[t][r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r + 1], k) * uu.y);
                        acc[t][r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r + 2], k) * uu.z);
                        acc[t][r].add(__builtin_ldexpf((float)(int32_t)iv[4 * r + 3], k) * uu.w);
                    } else {
                        // FP32 row sum inside the block; the power-of-two
                        // block scale is applied once to that sum
                        float p = (float)(int32_t)iv[4 * r] * uu.x;
                        p = __builtin_fmaf((float)(int32_t)iv[4 * r + 1], uu.y, p);
                        p = __builtin_fmaf((float)(int32_t)iv[4 * r + 2], uu.z, p);
                        p = __builtin_fmaf((float)(int32_t)iv[4 * r + 3], uu.w, p);
                        acc[t][r].add(__builtin_ldexpf(p, emax - 30));
                    }
                }
            }
        }
    }

    // reduce across the 64 lanes of each wave, then across the 4 waves
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int mask = 32; mask >= 1; mask >>= 1)
                acc[t][r].merge_from_lane(mask);
            if (lane == 0)
                red[wave][4 * t + r] = acc[t][r].value();
        }
    __syncthreads();
    if (threadIdx.x < (uint32_t)(4 * nr)) {
        const int k = threadIdx.x;
        double s = red[0][k];
#pragma unroll
        for (int q = 1; q < kThreads / 64; ++q)
            s += red[q][k];
        const uint32_t out_row = (bi0 - bi_begin) * 4 + k;
        if (nslab == 1)
            y[out_row] = (float)s;
        else
            part[(uint64_t)slab * ((bi_end - bi_begin) * 4) + out_row] = s;
    }
}

__global__ void __launch_bounds__(kThreads) reduce_slabs_kernel(const double* __restrict__ part, uint32_t nrows,
                                                                uint32_t nslab, float* __restrict__ y)
{
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= nrows)
        return;
    double s = 0.0;
    for (uint32_t k = 0; k < nslab; ++k)
        s += part[(uint64_t)k * nrows + i];
    y[i] = (float)s;
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
    const uint64_t nb = (uint64_t)(rows / 4) * (cols / 4);
    hipLaunchKernelGGL(decode_matrix_kernel<NW>, dim3(grid_for(nb, 65536)), dim3(kThreads), 0, st, s, cols / 4,
                       nb, cols, out);
    return hipGetLastError();
}

template <int NW>
hipError_t launch_encode(const float* M, uint32_t rows, uint32_t cols, uint32_t* s, uint32_t* bad, hipStream_t st)
{
    const uint64_t nb = (uint64_t)(rows / 4) * (cols / 4);
    hipLaunchKernelGGL(encode_kernel<NW>, dim3(grid_for(nb, 65536)), dim3(kThreads), 0, st, M, cols / 4, cols, nb,
                       s, bad);
    return hipGetLastError();
}

template <int NW, int TR, typename Acc>
hipError_t launch_gemv_t(const GemvPlan& pl, const uint32_t* s, const float* u, float* y, double* part,
                         hipStream_t st)
{
    hipLaunchKernelGGL((gemv_kernel<NW, TR, Acc>), dim3(pl.ntiles * pl.nslab), dim3(kThreads), 0, st, s, u, y, part,
                       pl.nbc, pl.bi_begin, pl.bi_end, pl.slab_bc, pl.nslab);
    return hipGetLastError();
}

template <int NW>
hipError_t launch_gemv(const GemvPlan& pl, AccMode mode, const uint32_t* s, const float* u, float* y, double* part,
                       hipStream_t st)
{
    hipError_t e = mode == AccMode::TwoSum  ? launch_gemv_t<NW, kGemvTileRows, TwoSumAcc>(pl, s, u, y, part, st)
                   : mode == AccMode::PaperMp ? launch_gemv_t<NW, kGemvTileRows, PaperMpAcc>(pl, s, u, y, part, st)
                                              : launch_gemv_t<NW, kGemvTileRows, Fp64Acc>(pl, s, u, y, part, st);
    if (e != hipSuccess || pl.nslab == 1)
        return e;
    const uint32_t nrows = (pl.bi_end - pl.bi_begin) * 4;
    hipLaunchKernelGGL(reduce_slabs_kernel, dim3(grid_for(nrows)), dim3(kThreads), 0, st, part, nrows, pl.nslab, y);
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

} // namespace nwN
} // namespace wh
