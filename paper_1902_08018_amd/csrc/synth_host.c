/*
 * synth_host.c -- seeded synthetic inputs (host side).
 *
 * Stand-in for the paper's deformation matrices C_d and thermal vectors S_k
 * (Sec. 2.1, Eq. 2), which are not public: a dense response matrix over two
 * unit-spaced 2-D lattices, M[i,j] = exp(-|p_i - q_j| / ell) + sigma * z_ij,
 * rounded once to FP32, and dose vectors u_j uniform on [0, 1).
 *
 * Holds none of the codec or GEMV arithmetic.  The same definitions are
 * implemented for the GPU in synth_dev.hip; both must produce identical bits
 * (integer hashing, FP64 multiply/add with no contraction, one RNE to FP32;
 * the exp table is computed here with the host libm and handed to both).
 *
 * Counter-based randomness: the SplitMix64 output function (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * applied to key(seed, stream) + (k + 1) * 0x9E3779B97F4A7C15.
 * Normal noise: Irwin-Hall sum of twelve 24-bit uniforms minus 6 (mean 0,
 * variance 1, support [-6, 6]).
 */
#include <math.h>
#include <stdint.h>

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t whs_hash(uint64_t seed, uint32_t stream, uint64_t k)
{
    uint64_t key = mix64((seed << 8) | (stream & 0xFFu));
    return mix64(key + (k + 1) * 0x9E3779B97F4A7C15ull);
}

/* exp(-sqrt(dx^2 + dy^2) / ell) for dx in [0, g), dy in [0, ndy);
 * table[dy * g + dx]. */
void whs_kernel_table(uint32_t g, uint32_t ndy, double ell, double *table)
{
    for (uint32_t dy = 0; dy < ndy; dy++)
        for (uint32_t dx = 0; dx < g; dx++)
            table[(uint64_t)dy * g + dx] = exp(-sqrt((double)dx * dx + (double)dy * dy) / ell);
}

/* Irwin-Hall(12) normal deviate for matrix element number `lin`. */
static double noise(uint64_t seed, uint64_t lin)
{
    int64_t acc = 0;
    for (int t = 0; t < 6; t++) {
        uint64_t h = whs_hash(seed, 0, 6 * lin + (uint64_t)t);
        acc += (int64_t)(h >> 40) + (int64_t)((h >> 16) & 0xFFFFFFu);
    }
    return (double)(acc - 6 * (int64_t)(1 << 24)) * (1.0 / 16777216.0);
}

static uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

/* Rows [r0, r1) of the cols-wide matrix into out[(r1 - r0) * cols]. */
void whs_matrix_rows(uint64_t seed, uint32_t g, uint32_t cols, double sigma, const double *table, uint32_t r0,
                     uint32_t r1, float *out)
{
    for (uint32_t i = r0; i < r1; i++) {
        for (uint32_t j = 0; j < cols; j++) {
            uint32_t dx = absdiff(i % g, j % g), dy = absdiff(i / g, j / g);
            double t = sigma * noise(seed, (uint64_t)i * cols + j);
            double v = table[(uint64_t)dy * g + dx] + t;
            out[(uint64_t)(i - r0) * cols + j] = (float)v;
        }
    }
}

/* n values uniform on [0, 1) with 24 random bits (exact in FP32): element
 * k of the vector is (hash(seed, stream, offset + k) >> 40) * 2^-24. */
void whs_uniform(uint64_t seed, uint32_t stream, uint64_t offset, uint64_t n, float *out)
{
    for (uint64_t k = 0; k < n; k++)
        out[k] = (float)(whs_hash(seed, stream, offset + k) >> 40) * (1.0f / 16777216.0f);
}
