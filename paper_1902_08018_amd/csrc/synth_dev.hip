// synth_dev.hip -- seeded synthetic inputs generated on the GPU.
//
// Device twin of synth_host.c for matrices too large to build on the host
// (65536 x 65536 FP32 is 17 GB).  Same definitions, same bits: SplitMix64
// output function over a counter, Irwin-Hall(12) noise from twelve 24-bit
// uniforms, FP64 multiply then add (this file is compiled with
// -ffp-contract=off so they are never fused), one RNE conversion to FP32.
// The exp table is computed on the host and passed in.
//
// Holds none of the codec or GEMV arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t hash_at(uint64_t key, uint64_t k)
{
    return mix64(key + (k + 1) * 0x9E3779B97F4A7C15ull);
}

uint64_t host_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t stream_key(uint64_t seed, uint32_t stream) { return host_mix64((seed << 8) | (stream & 0xFFu)); }

__global__ void __launch_bounds__(256) matrix_rows_kernel(uint64_t key, uint32_t g, uint32_t cols, double sigma,
                                                          const double* __restrict__ table, uint32_t r0,
                                                          uint64_t count, float* __restrict__ out)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
        uint32_t i = r0 + (uint32_t)(e / cols);
        uint32_t j = (uint32_t)(e % cols);
        uint64_t lin = (uint64_t)i * cols + j;
        int64_t acc = 0;
#pragma unroll
        for (int t = 0; t < 6; t++) {
            uint64_t h = hash_at(key, 6 * lin + (uint64_t)t);
            acc += (int64_t)(h >> 40) + (int64_t)((h >> 16) & 0xFFFFFFu);
        }
        double z = (double)(acc - 6 * (int64_t)(1 << 24)) * (1.0 / 16777216.0);
        uint32_t ia = i % g, ja = j % g, ib = i / g, jb = j / g;
        uint32_t dx = ia > ja ? ia - ja : ja - ia;
        uint32_t dy = ib > jb ? ib - jb : jb - ib;
        double t = sigma * z;
        double v = table[(uint64_t)dy * g + dx] + t;
        out[e] = (float)v;
    }
}

__global__ void __launch_bounds__(256) uniform_kernel(uint64_t key, uint64_t offset, uint64_t n,
                                                      float* __restrict__ out)
{
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        out[k] = (float)(hash_at(key, offset + k) >> 40) * (1.0f / 16777216.0f);
}

unsigned grid_for(uint64_t n)
{
    uint64_t blocks = (n + 255) / 256;
    return (unsigned)(blocks < 65536 ? (blocks ? blocks : 1) : 65536);
}

}  // namespace

// Rows [r0, r1) of the cols-wide matrix into d_out (device, (r1-r0)*cols
// floats).  d_table: device copy of the host exp table (see synth_host.c).
extern "C" int whs_dev_matrix_rows(uint64_t seed, uint32_t g, uint32_t cols, double sigma, const double* d_table,
                                   uint32_t r0, uint32_t r1, float* d_out, void* stream)
{
    if (r1 < r0 || g == 0 || cols == 0)
        return -1;
    uint64_t count = (uint64_t)(r1 - r0) * cols;
    if (count == 0)
        return 0;
    hipLaunchKernelGGL(matrix_rows_kernel, dim3(grid_for(count)), dim3(256), 0, (hipStream_t)stream,
                       stream_key(seed, 0), g, cols, sigma, d_table, r0, count, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}

extern "C" int whs_dev_uniform(uint64_t seed, uint32_t stream_id, uint64_t offset, uint64_t n, float* d_out,
                               void* stream)
{
    if (n == 0)
        return 0;
    hipLaunchKernelGGL(uniform_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream,
                       stream_key(seed, stream_id), offset, n, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -6;
}
