// dense_kernels.hip -- GEMV over dense matrices stored in reduced precision,
// and the quantisers that produce them.
//
// The paper's GEMV multiplies FP32 values and reduces in FP64 (Sec. 4.4,
// Fig. 7).  Here the matrix may be held in FP32, FP16, BF16 (row-major) or
// OCP FP8 e4m3 with one FP32 scale per 4x4 block; every format is widened to
// FP32 in registers, multiplied in FP32, summed in FP32 over a short run
// (4 or 8 values), then accumulated across runs in FP64 or compensated FP32.
// These kernels only stream the matrix once; they are HBM-bound.
//
// Row-major formats: one workgroup (256 lanes) per (tile of 8 rows, column
// slab); a lane reads 16 bytes of each of the 8 rows per step (4 FP32 or
// 8 FP16/BF16 values), so one step of a workgroup reads 8 contiguous 4 KiB
// runs.  FP8 block-scaled: one lane per 4x4 block (16 code bytes + 4 scale
// bytes), 4 block-rows per tile, like the compressed path.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "wh_ctx.hpp"
#include "wh_internal.hpp"

namespace wh {
namespace {

constexpr int kThreads = 256;
constexpr int kDenseRows = 8;

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

struct AccF64 {
    double s;
    __device__ __forceinline__ void zero() { s = 0.0; }
    __device__ __forceinline__ void add(float p) { s += (double)p; }
    __device__ __forceinline__ double value() const { return s; }
    __device__ __forceinline__ void merge_from_lane(int mask) { s += __shfl_xor(s, mask, 64); }
};

struct AccTwoSum {
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

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }

// Per-format loader: one lane-step = kElems consecutive values of a row,
// one 16-byte load kept raw until each value is multiplied (widening all of
// them at once would hold kElems FP32 registers per row).
struct F32Fmt {
    static constexpr int kElems = 4;
    static constexpr int kBytes = 4;
    typedef f32x4 Raw;
    __device__ __forceinline__ static Raw load(const void* base, uint64_t elem)
    {
        return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(base) + elem / 4);
    }
    __device__ __forceinline__ static float get(const Raw& x, int k) { return x[k]; }
};

template <bool BF>
struct Half16Fmt {
    static constexpr int kElems = 8;
    static constexpr int kBytes = 2;
    typedef u16x8 Raw;
    __device__ __forceinline__ static Raw load(const void* base, uint64_t elem)
    {
        return __builtin_nontemporal_load(reinterpret_cast<const u16x8*>(base) + elem / 8);
    }
    __device__ __forceinline__ static float get(const Raw& x, int k)
    {
        return BF ? bf16_to_f32(x[k]) : f16_to_f32(x[k]);
    }
};

// Reduce TRxlanes accumulators and write y (single slab) or FP64 partials.
template <int NROW, typename Acc>
__device__ __forceinline__ void finish_rows(Acc (&acc)[NROW], uint32_t nrows_here, uint32_t out_row0,
                                            uint32_t nrows_out, uint32_t slab, uint32_t nslab, float* y,
                                            double* part)
{
    __shared__ double red[kThreads / 64][NROW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < NROW; ++t) {
#pragma unroll
        for (int mask = 32; mask >= 1; mask >>= 1)
            acc[t].merge_from_lane(mask);
        if (lane == 0)
            red[wave][t] = acc[t].value();
    }
    __syncthreads();
    if (threadIdx.x < nrows_here) {
        const int k = threadIdx.x;
        double s = red[0][k];
#pragma unroll
        for (int q = 1; q < kThreads / 64; ++q)
            s += red[q][k];
        if (nslab == 1)
            y[out_row0 + k] = (float)s;
        else
            part[(uint64_t)slab * nrows_out + out_row0 + k] = s;
    }
}

// Row-major dense GEMV.  Steps of kElems values; step_cols = cols / kElems.
template <typename Fmt, typename Acc>
__global__ void __launch_bounds__(kThreads) dense_rowmajor_kernel(const void* __restrict__ M,
                                                                  const float* __restrict__ u, float* __restrict__ y,
                                                                  double* __restrict__ part, uint32_t cols,
                                                                  uint32_t row_begin, uint32_t row_end,
                                                                  uint32_t slab_steps, uint32_t nslab)
{
    constexpr int E = Fmt::kElems;
    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t r0 = row_begin + tile * kDenseRows;
    const uint32_t nr = row_end - r0 < (uint32_t)kDenseRows ? row_end - r0 : (uint32_t)kDenseRows;
    const uint32_t nsteps = cols / E;
    const uint32_t s0 = slab * slab_steps;
    const uint32_t s1 = s0 + slab_steps < nsteps ? s0 + slab_steps : nsteps;

    Acc acc[kDenseRows];
#pragma unroll
    for (int t = 0; t < kDenseRows; ++t)
        acc[t].zero();

    for (uint32_t step = s0 + threadIdx.x; step < s1; step += kThreads) {
        float uu[E];
#pragma unroll
        for (int k = 0; k < E; k += 4) {
            const f32x4 x = reinterpret_cast<const f32x4*>(u)[(step * E + k) / 4];
            uu[k] = x.x;
            uu[k + 1] = x.y;
            uu[k + 2] = x.z;
            uu[k + 3] = x.w;
        }
        typename Fmt::Raw m[kDenseRows];
#pragma unroll
        for (int t = 0; t < kDenseRows; ++t)
            if ((uint32_t)t < nr)
                m[t] = Fmt::load(M, (uint64_t)(r0 + t) * cols + (uint64_t)step * E);
#pragma unroll
        for (int t = 0; t < kDenseRows; ++t) {
            if ((uint32_t)t < nr) {
#pragma unroll
                for (int g = 0; g < E; g += 4) {
                    float p = Fmt::get(m[t], g) * uu[g];
                    p = __builtin_fmaf(Fmt::get(m[t], g + 1), uu[g + 1], p);
                    p = __builtin_fmaf(Fmt::get(m[t], g + 2), uu[g + 2], p);
                    p = __builtin_fmaf(Fmt::get(m[t], g + 3), uu[g + 3], p);
                    acc[t].add(p);
                }
            }
        }
    }
    finish_rows<kDenseRows>(acc, nr, r0 - row_begin, row_end - row_begin, slab, nslab, y, part);
}

// Fig. 7 on a dense FP32 matrix: every FP32 product added to the FP64 sum.
__global__ void __launch_bounds__(kThreads) dense_f32_paper_mp_kernel(const float* __restrict__ M,
                                                                      const float* __restrict__ u,
                                                                      float* __restrict__ y,
                                                                      double* __restrict__ part, uint32_t cols,
                                                                      uint32_t row_begin, uint32_t row_end,
                                                                      uint32_t slab_steps, uint32_t nslab)
{
    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t r0 = row_begin + tile * kDenseRows;
    const uint32_t nr = row_end - r0 < (uint32_t)kDenseRows ? row_end - r0 : (uint32_t)kDenseRows;
    const uint32_t nsteps = cols / 4;
    const uint32_t s0 = slab * slab_steps;
    const uint32_t s1 = s0 + slab_steps < nsteps ? s0 + slab_steps : nsteps;
    AccF64 acc[kDenseRows];
#pragma unroll
    for (int t = 0; t < kDenseRows; ++t)
        acc[t].zero();
    for (uint32_t step = s0 + threadIdx.x; step < s1; step += kThreads) {
        const f32x4 uu = reinterpret_cast<const f32x4*>(u)[step];
#pragma unroll
        for (int t = 0; t < kDenseRows; ++t) {
            if ((uint32_t)t < nr) {
                const f32x4 m = reinterpret_cast<const f32x4*>(M + (uint64_t)(r0 + t) * cols)[step];
                acc[t].add(m.x * uu.x);
                acc[t].add(m.y * uu.y);
                acc[t].add(m.z * uu.z);
                acc[t].add(m.w * uu.w);
            }
        }
    }
    finish_rows<kDenseRows>(acc, nr, r0 - row_begin, row_end - row_begin, slab, nslab, y, part);
}

// --------------------------------------------------------- FP8 e4m3 + scale
// Codes: block b = bi*(cols/4) + bj at bytes [16b, 16b+16), value v = 4r + c
// in byte v.  Scales: FP32 at bytes 16*nb + 4b.  Value = decode(code) * scale.
__device__ __forceinline__ void fp8x4_to_f32(uint32_t w, float (&o)[4])
{
    // OCP e4m3 (gfx950 native conversion), two bytes per instruction
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
    o[0] = lo[0];
    o[1] = lo[1];
    o[2] = hi[0];
    o[3] = hi[1];
}

constexpr int kFp8TileRows = 4;

template <typename Acc>
__global__ void __launch_bounds__(kThreads) fp8bs_kernel(const uint8_t* __restrict__ codes,
                                                         const float* __restrict__ scales,
                                                         const float* __restrict__ u, float* __restrict__ y,
                                                         double* __restrict__ part, uint32_t nbc, uint32_t bi_begin,
                                                         uint32_t bi_end, uint32_t slab_bc, uint32_t nslab)
{
    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t bi0 = bi_begin + tile * kFp8TileRows;
    const uint32_t nr = bi_end - bi0 < (uint32_t)kFp8TileRows ? bi_end - bi0 : (uint32_t)kFp8TileRows;
    const uint32_t bc0 = slab * slab_bc;
    const uint32_t bc1 = bc0 + slab_bc < nbc ? bc0 + slab_bc : nbc;
    Acc acc[kFp8TileRows * 4];
#pragma unroll
    for (int t = 0; t < kFp8TileRows * 4; ++t)
        acc[t].zero();
    for (uint32_t bj = bc0 + threadIdx.x; bj < bc1; bj += kThreads) {
        const f32x4 uu = reinterpret_cast<const f32x4*>(u)[bj];
        u32x4 q[kFp8TileRows];
        float sc[kFp8TileRows];
#pragma unroll
        for (int t = 0; t < kFp8TileRows; ++t) {
            if ((uint32_t)t < nr) {
                const uint64_t b = (uint64_t)(bi0 + t) * nbc + bj;
                q[t] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(codes) + b);
                sc[t] = __builtin_nontemporal_load(scales + b);
            }
        }
#pragma unroll
        for (int t = 0; t < kFp8TileRows; ++t) {
            if ((uint32_t)t < nr) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float f[4];
                    fp8x4_to_f32(q[t][r], f);
                    float p = f[0] * uu.x;
                    p = __builtin_fmaf(f[1], uu.y, p);
                    p = __builtin_fmaf(f[2], uu.z, p);
                    p = __builtin_fmaf(f[3], uu.w, p);
                    acc[4 * t + r].add(p * sc[t]);
                }
            }
        }
    }
    finish_rows<kFp8TileRows * 4>(acc, 4 * nr, (bi0 - bi_begin) * 4, (bi_end - bi_begin) * 4, slab, nslab, y,
                                  part);
}

__global__ void __launch_bounds__(kThreads) reduce_partials_kernel(const double* __restrict__ part, uint32_t nrows,
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

// ----------------------------------------------------------- quantisers
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__global__ void __launch_bounds__(kThreads) quant_half_kernel(const float* __restrict__ M, uint64_t n, int bf,
                                                              uint16_t* __restrict__ out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const float f = M[i];
        out[i] = bf ? f32_to_bf16_rne(f) : __half_as_ushort(__float2half_rn(f));
    }
}

// Round-to-nearest-even of x (|x| <= 448 after scaling, finite) to an OCP
// e4m3 code: bias 7, 3 mantissa bits, subnormals below 2^-6, max 448.
__device__ __forceinline__ uint32_t f32_to_e4m3_rne(float x)
{
    const uint32_t sign = (__float_as_uint(x) >> 31) << 7;
    float a = __builtin_fabsf(x);
    if (a >= 448.0f)
        return sign | 0x7Eu; // saturate to the largest finite value
    // quantum of the binade of a (subnormal quantum 2^-9 below 2^-6)
    int e;
    (void)__builtin_frexpf(a, &e); // a in [2^(e-1), 2^e)
    int qexp = (e - 1) - 3;
    if (qexp < -9)
        qexp = -9;
    // a / quantum is exact (power-of-two scaling); rint() rounds half to even
    const float k = __builtin_rintf(__builtin_ldexpf(a, -qexp));
    const float r = __builtin_ldexpf(k, qexp); // rounded magnitude (may step to the next binade)
    if (r == 0.0f)
        return 0u; // a value that rounds to zero has code 0 (never -0)
    int re;
    (void)__builtin_frexpf(r, &re);
    const int E = (re - 1) + 7; // biased exponent if normal
    if (E <= 0) { // subnormal: value = m * 2^-9
        const uint32_t m = (uint32_t)__builtin_ldexpf(r, 9);
        return sign | m;
    }
    const uint32_t m = (uint32_t)__builtin_ldexpf(r, -(re - 1) + 3) - 8u; // 1.mmm * 8 - 8
    return sign | ((uint32_t)E << 3) | m;
}

__global__ void __launch_bounds__(kThreads) quant_fp8bs_kernel(const float* __restrict__ M, uint32_t nbc,
                                                               uint32_t cols, uint64_t nb, uint8_t* __restrict__ codes,
                                                               float* __restrict__ scales)
{
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < nb; b += stride) {
        const uint64_t bi = b / nbc, bj = b % nbc;
        float f[16];
        float amax = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const f32x4 v = *reinterpret_cast<const f32x4*>(M + (4 * bi + r) * cols + 4 * bj);
            f[4 * r] = v.x;
            f[4 * r + 1] = v.y;
            f[4 * r + 2] = v.z;
            f[4 * r + 3] = v.w;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)
            amax = __builtin_fmaxf(amax, __builtin_fabsf(f[v]));
        u32x4 q = {0u, 0u, 0u, 0u};
        float s = 0.0f;
        if (amax > 0.0f) {
            s = __fdiv_rn(amax, 448.0f);
            const float inv = __fdiv_rn(448.0f, amax);
#pragma unroll
            for (int v = 0; v < 16; ++v)
                q[v >> 2] |= f32_to_e4m3_rne(__fmul_rn(f[v], inv)) << (8 * (v & 3));
        }
        reinterpret_cast<u32x4*>(codes)[b] = q;
        scales[b] = s;
    }
}

// Read-only streaming probe: every 16-byte vector of the buffer is loaded
// once (non-temporal, 4 vectors in flight per lane per step, grid-stride)
// and folded by XOR; one atomic XOR per workgroup publishes the fold.  Its
// time is the practical HBM read ceiling of the device for a stream that is
// read once and not written, the access pattern of the compressed GEMV.
__global__ void __launch_bounds__(kThreads) stream_read_kernel(const u32x4* __restrict__ buf, uint64_t nvec,
                                                               uint32_t* __restrict__ out)
{
    __shared__ uint32_t red[kThreads / 64];
    constexpr uint64_t kUnroll = 4;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    uint32_t x = 0;
    uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < nvec; i += kUnroll * stride) {
        u32x4 v[kUnroll];
#pragma unroll
        for (uint64_t k = 0; k < kUnroll; ++k)
            v[k] = __builtin_nontemporal_load(buf + i + k * stride);
#pragma unroll
        for (uint64_t k = 0; k < kUnroll; ++k)
            x ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
    }
    for (; i < nvec; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(buf + i);
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    for (int m = 32; m >= 1; m >>= 1)
        x ^= (uint32_t)__shfl_xor((int)x, m, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kThreads / 64; ++w)
            t ^= red[w];
        atomicXor(out, t);
    }
}

unsigned grid_for(uint64_t items, unsigned cap = 65536)
{
    uint64_t g = (items + kThreads - 1) / kThreads;
    if (g == 0)
        g = 1;
    return (unsigned)(g < cap ? g : cap);
}

// Column slabs so that (row tiles x slabs) fills the chip several times.
uint32_t choose_slabs(uint32_t ntiles, uint32_t nsteps, int num_cus, uint32_t& slab_steps)
{
    const uint64_t want = (uint64_t)(num_cus > 0 ? num_cus : 256) * 8;
    const uint32_t max_slabs = (nsteps + kThreads - 1) / kThreads;
    uint32_t nslab = ntiles ? (uint32_t)((want + ntiles - 1) / ntiles) : 1;
    if (nslab < 1)
        nslab = 1;
    if (nslab > max_slabs)
        nslab = max_slabs ? max_slabs : 1;
    slab_steps = (nsteps + nslab - 1) / nslab;
    slab_steps = (slab_steps + kThreads - 1) / kThreads * kThreads;
    if (slab_steps == 0)
        slab_steps = kThreads;
    nslab = (nsteps + slab_steps - 1) / slab_steps;
    return nslab < 1 ? 1 : nslab;
}

template <typename Fmt>
hipError_t launch_rowmajor(const void* M, AccMode mode, const float* u, float* y, double* part, uint32_t cols,
                           uint32_t r0, uint32_t r1, uint32_t ntiles, uint32_t slab_steps, uint32_t nslab,
                           hipStream_t st)
{
    const dim3 grid(ntiles * nslab);
    if (mode == AccMode::TwoSum)
        hipLaunchKernelGGL((dense_rowmajor_kernel<Fmt, AccTwoSum>), grid, dim3(kThreads), 0, st, M, u, y, part, cols,
                           r0, r1, slab_steps, nslab);
    else
        hipLaunchKernelGGL((dense_rowmajor_kernel<Fmt, AccF64>), grid, dim3(kThreads), 0, st, M, u, y, part, cols, r0,
                           r1, slab_steps, nslab);
    return hipGetLastError();
}

} // namespace

wh_status dense_gemv_dispatch(wh_ctx* ctx, const Matrix& mat, AccMode mode, const float* d_u, float* d_y,
                              uint32_t row_begin, uint32_t row_end, hipStream_t st)
{
    const uint32_t cols = mat.desc.cols, nrows = row_end - row_begin;
    const int fmt = mat.desc.fmt;
    if (mode == AccMode::PaperMp && fmt != WH_FMT_F32)
        return WH_ERR_FORMAT;
    hipError_t e = hipSuccess;
    uint32_t nslab = 1;
    if (fmt == WH_FMT_FP8E4M3_BS4) {
        GemvPlan pl = block_slab_plan(cols, row_begin, row_end, ctx->num_cus, kThreads, kFp8TileRows);
        nslab = pl.nslab;
        double* part = nullptr;
        if (nslab > 1) {
            wh_status s2 = ensure_partials(ctx, (size_t)nslab * nrows, st);
            if (s2 != WH_OK)
                return s2;
            part = ctx->part;
        }
        const uint64_t nb = (uint64_t)(mat.desc.rows / 4) * (cols / 4);
        const uint8_t* codes = static_cast<const uint8_t*>(mat.dptr);
        const float* scales = reinterpret_cast<const float*>(codes + nb * 16);
        const uint32_t ntiles = (pl.bi_end - pl.bi_begin + kFp8TileRows - 1) / kFp8TileRows;
        const dim3 grid(ntiles * nslab);
        if (mode == AccMode::TwoSum)
            hipLaunchKernelGGL(fp8bs_kernel<AccTwoSum>, grid, dim3(kThreads), 0, st, codes, scales, d_u, d_y, part,
                               pl.nbc, pl.bi_begin, pl.bi_end, pl.slab_bc, nslab);
        else
            hipLaunchKernelGGL(fp8bs_kernel<AccF64>, grid, dim3(kThreads), 0, st, codes, scales, d_u, d_y, part,
                               pl.nbc, pl.bi_begin, pl.bi_end, pl.slab_bc, nslab);
        e = hipGetLastError();
        if (e == hipSuccess && nslab > 1) {
            hipLaunchKernelGGL(reduce_partials_kernel, dim3(grid_for(nrows)), dim3(kThreads), 0, st, part, nrows,
                               nslab, d_y);
            e = hipGetLastError();
        }
        return device_error(ctx, part ? partials_release(ctx, st, e) : e);
    }
    const int elems = fmt == WH_FMT_F32 ? 4 : 8;
    if (cols % elems)
        return WH_ERR_SHAPE; // FP16/BF16 rows are read 8 values at a time
    const uint32_t ntiles = (nrows + kDenseRows - 1) / kDenseRows;
    uint32_t slab_steps = 0;
    nslab = choose_slabs(ntiles, cols / elems, ctx->num_cus, slab_steps);
    double* part = nullptr;
    if (nslab > 1) {
        wh_status s2 = ensure_partials(ctx, (size_t)nslab * nrows, st);
        if (s2 != WH_OK)
            return s2;
        part = ctx->part;
    }
    switch (fmt) {
    case WH_FMT_F32:
        if (mode == AccMode::PaperMp) {
            hipLaunchKernelGGL(dense_f32_paper_mp_kernel, dim3(ntiles * nslab), dim3(kThreads), 0, st,
                               static_cast<const float*>(mat.dptr), d_u, d_y, part, cols, row_begin, row_end,
                               slab_steps, nslab);
            e = hipGetLastError();
        } else {
            e = launch_rowmajor<F32Fmt>(mat.dptr, mode, d_u, d_y, part, cols, row_begin, row_end, ntiles, slab_steps,
                                        nslab, st);
        }
        break;
    case WH_FMT_F16:
        e = launch_rowmajor<Half16Fmt<false>>(mat.dptr, mode, d_u, d_y, part, cols, row_begin, row_end, ntiles,
                                              slab_steps, nslab, st);
        break;
    case WH_FMT_BF16:
        e = launch_rowmajor<Half16Fmt<true>>(mat.dptr, mode, d_u, d_y, part, cols, row_begin, row_end, ntiles,
                                             slab_steps, nslab, st);
        break;
    default:
        return WH_ERR_FORMAT;
    }
    if (e == hipSuccess && nslab > 1) {
        hipLaunchKernelGGL(reduce_partials_kernel, dim3(grid_for(nrows)), dim3(kThreads), 0, st, part, nrows, nslab,
                           d_y);
        e = hipGetLastError();
    }
    return device_error(ctx, part ? partials_release(ctx, st, e) : e);
}

} // namespace wh

extern "C" wh_status wh_quantize(wh_ctx* ctx, const float* d_M, uint32_t rows, uint32_t cols, int32_t fmt,
                                 void* d_out, void* stream)
{
    using namespace wh;
    if (!ctx)
        return WH_ERR_INVALID;
    if (ctx->failed.load())
        return WH_ERR_DEVICE;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return WH_ERR_DEVICE;
    if (!d_M || !d_out || !aligned(d_M, 16) || !aligned(d_out, 16))
        return WH_ERR_INVALID;
    if (rows == 0 || cols == 0 || rows % 4 || cols % 4)
        return WH_ERR_SHAPE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t n = (uint64_t)rows * cols;
    try {
        switch (fmt) {
        case WH_FMT_F16:
        case WH_FMT_BF16:
            hipLaunchKernelGGL(quant_half_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, d_M, n,
                               fmt == WH_FMT_BF16 ? 1 : 0, static_cast<uint16_t*>(d_out));
            return device_error(ctx, hipGetLastError());
        case WH_FMT_FP8E4M3_BS4: {
            const uint64_t nb = n / 16;
            uint8_t* codes = static_cast<uint8_t*>(d_out);
            hipLaunchKernelGGL(quant_fp8bs_kernel, dim3(grid_for(nb)), dim3(kThreads), 0, st, d_M, cols / 4, cols, nb,
                               codes, reinterpret_cast<float*>(codes + nb * 16));
            return device_error(ctx, hipGetLastError());
        }
        default:
            return WH_ERR_FORMAT;
        }
    } catch (...) {
        return WH_ERR_INVALID;
    }
}

extern "C" wh_status wh_stream_read(wh_ctx* ctx, const void* d_buf, uint64_t nbytes, uint32_t* d_out, void* stream)
{
    using namespace wh;
    if (!ctx)
        return WH_ERR_INVALID;
    if (ctx->failed.load())
        return WH_ERR_DEVICE;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return WH_ERR_DEVICE;
    if (!d_buf || !d_out || !aligned(d_buf, 16) || nbytes % 16 != 0)
        return WH_ERR_INVALID;
    const uint64_t nvec = nbytes / 16;
    if (nvec == 0)
        return WH_OK;
    // about 8 workgroups of 256 lanes per CU, each lane with 4 loads in flight
    const uint64_t want = (nvec + kThreads - 1) / kThreads;
    const uint64_t cap = (uint64_t)(ctx->num_cus > 0 ? ctx->num_cus : 256) * 8;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(kThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const u32x4*>(d_buf), nvec, d_out);
    return device_error(ctx, hipGetLastError());
}
