// whz_var.hip -- the variable-rate WHZ1 modes: fixed precision and fixed
// accuracy (the paper's zfp modes besides fixed rate, Sec. 4.3, Table 2).
//
// Code: the fixed-rate block code with no bit budget.  A nonzero block codes
// bit planes 31 down to 32 - P and ends there:
//   fixed precision  P = the precision (1..32) for every block;
//   fixed accuracy   P = clamp(emax - minexp + 7, 0, 32) for the tolerance
//                    2^minexp, which keeps every value within the tolerance
//                    wherever P is not clamped at 32 (emax - minexp <= 25).
// Blocks follow one another with no padding, block rows in order.  The index
// (in front of the code) holds the bit offset of every 32nd block of each
// block row, so a lane can start at a group of 32 blocks and walk it.
//
// Storage: [index: ceil(rows/4) x ceil(ceil(cols/4)/32) uint64][code bytes].
//
// Decoding: one lane per group of 32 blocks, the blocks in sequence; the
// lanes of a wave run the bit planes in lockstep (as the fixed-rate decoder),
// each with its own lowest plane.  Before each block a lane brings the next
// words of its code into its own LDS ring (word-major, as the fixed-rate
// staging; only the 16-byte pieces not already there), so the decoder's
// window reads are LDS reads, not chains of dependent global loads.  The fused GEMV gives 1 to 8 lanes (groups) to a block row
// and multiplies each block's exactly decoded values by u.  The encoder runs
// on the host (the paper encodes offline, Sec. 4.3).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "../../include/wh.h"
#include "whz_device.hpp"
#include "wh_ctx.hpp"
#include "wh_internal.hpp"

namespace wh {

namespace {

// Workgroup sizes: 256 lanes, or for the fused GEMV 1024 from 2^18 lanes of
// work up (16 waves per CU share one section table, where LDS holds only two
// 256-lane workgroups, 8 waves).
constexpr int kVarThreadsSmall = 256, kVarThreadsLarge = 1024;
constexpr uint64_t kVarLargeFrom = 1ull << 18;

__device__ const SectionTable g_var_section_table{};

template <int T>
__device__ __forceinline__ void load_table(uint32_t* tab)
{
    for (int i = threadIdx.x; i < kSecEntries; i += T)
        tab[i] = g_var_section_table.e[i];
    __syncthreads();
}

// Word i of a lane's code view (g = the word holding its group's first bit,
// lim = the words from there to the end of the code); zero past the end.
__device__ __forceinline__ uint32_t vword(const uint32_t* __restrict__ g, uint32_t lim, uint32_t i)
{
    return i < lim ? g[i] : 0u;
}

// 32 code bits from bit position pos of the view.
__device__ __forceinline__ uint32_t vwindow(const uint32_t* __restrict__ g, uint32_t lim, uint32_t pos)
{
    const uint32_t q = pos >> 5;
    return funnel(vword(g, lim, q + 1), vword(g, lim, q), pos & 31u);
}

// A lane's code in LDS: a ring of kVarRing words, refilled 16 bytes at a
// time, so that each piece of the code is loaded from global memory once.
// A block of P planes takes at most 25 + 17 P bits: the 9-bit header, at
// most 16 verbatim bits a plane after the first, one ending group bit a
// plane, and across all planes at most 16 run-starting group bits and 16 run
// bits (a run passes each coefficient once).  With P <= 32, the start
// offset (< 32) and the last 32-bit window, every read stays below bit 632
// of the block's first word: 20 words hold any block.  Before a block the
// ring is filled through 24 words from the 16-byte boundary at or before
// that word (up to 3 words earlier): 6 pieces, of which the blocks before
// have already loaded all but the new ones.  One word after the ring
// mirrors its first, so that a window's two words are always adjacent.
constexpr uint32_t kVarRing = 24, kVarRow = kVarRing + 1;

// Reading a lane's code straight from global memory: two loads a window.
struct GlobalBits {
    const uint32_t* g;
    uint32_t lim;
    __device__ __forceinline__ uint32_t window(uint32_t pos) const { return vwindow(g, lim, pos); }
};

// Reading a block from a lane's ring at lw[k * T]: positions count from bit 0
// of the block's first 16-byte piece, which sits at word sb of the ring.  A
// window at or past word kVarRing - 1 reads the last word's slot (the word
// index is clamped), so a block that runs past 32 * (kVarRing - 1) bits
// must be decoded again from global memory.
template <int T>
struct StagedBits {
    const uint32_t* lw;
    uint32_t sb;
    __device__ __forceinline__ uint32_t window(uint32_t pos) const
    {
        uint32_t q = __builtin_elementwise_min(pos >> 5, kVarRing - 1u) + sb;
        q = __builtin_elementwise_min(q, q - kVarRing); // the ring's slot
        return funnel(lw[(q + 1) * T], lw[q * T], pos & 31u);
    }
};

// Planes coded for a block with exponent emax (mode 0: fixed precision,
// param = P; mode 1: fixed accuracy, param = minexp).
__host__ __device__ __forceinline__ int var_planes(int mode, int param, int emax)
{
    if (mode == 0)
        return param;
    const int p = emax - param + 7;
    return p < 0 ? 0 : (p > 32 ? 32 : p);
}

// Plane P of a block, all lanes in lockstep.  A lane whose lowest plane lo
// is above P reads zero bits: its plane word is zero, and its position and
// significance count stay put.  With no bit budget, the implied 1 at the end
// of a run is always coefficient 15's.
template <int P, typename Bits>
__device__ __forceinline__ void var_plane(const Bits& rd, const uint32_t* tab, uint32_t lo, uint32_t& pos,
                                          uint32_t& ns, uint32_t (&A)[16])
{
    const bool live = (uint32_t)P >= lo;
    const uint32_t w = live ? rd.window(pos) : 0u;
    const uint32_t xv = __builtin_amdgcn_ubfe(w, 0u, ns); // ns = nsig * kSecRow; v_bfe reads nsig
    uint32_t e = sec_lookup(tab, ns, __builtin_amdgcn_ubfe(w, ns, 8u));
    uint32_t acc = e;
    uint32_t at = add_nsig(pos, ns) + ent_used(e);
    ns += ent_adv(e) * (uint32_t)kSecRow;
    if (__any(ent_open(e))) {
        do {
            const uint32_t bits = live ? rd.window(at) : 0u;
            const uint32_t idx = ns + ent_next(e) + (bits & 0xFFu);
            e = tab[__builtin_elementwise_min(idx, (uint32_t)kSecDone)];
            acc |= e;
            at += ent_used(e);
            ns += ent_adv(e) * (uint32_t)kSecRow;
        } while (__any(ent_open(e)));
    }
    const uint32_t x = (acc & 0xFFFFu) | xv; // coefficient 15's implied 1 is in the table's ones
    if (live)
        pos = at;
    if constexpr (P >= 16)
        A[P - 16] = (x << 16) ^ kOddPlanes(P - 16);
    else
        A[P] ^= x;
}

template <int P, typename Bits>
__device__ __forceinline__ void var_planes_from(const Bits& rd, const uint32_t* tab, uint32_t lo, uint32_t& pos,
                                                uint32_t& ns, uint32_t (&A)[16])
{
    if constexpr (P >= 0) {
        if (!__any((uint32_t)P >= lo)) { // every lane is done: planes P..0 stay zero
            if constexpr (P >= 16) {
#pragma unroll
                for (int q = 0; q <= P - 16; ++q)
                    A[q] = kOddPlanes(q);
            }
            return;
        }
        var_plane<P>(rd, tab, lo, pos, ns, A);
        var_planes_from<P - 1>(rd, tab, lo, pos, ns, A);
    }
}

// Decode the block at pos (advanced past it) into its 16 transform
// coefficients (two's complement, local order 4r + c) and emax.  A lane with
// live == false decodes a zero block and does not move.  Returns whether the
// block is nonzero.
template <typename Bits>
__device__ __forceinline__ bool var_block_coeffs(const Bits& rd, const uint32_t* tab, int mode, int param, bool live,
                                                 uint32_t& pos, int& emax, uint32_t (&cf)[16])
{
    const uint32_t h = live ? rd.window(pos) : 0u;
    const bool nz = (h & 1u) != 0;
    emax = (int)((h >> 1) & 0xFFu) - 127;
    if (live)
        pos += nz ? 9u : 1u;
    const uint32_t lo = nz ? (uint32_t)(32 - var_planes(mode, param, emax)) : 32u;
    uint32_t ns = 0u; // nsig * kSecRow
    uint32_t A[16];
    var_planes_from<31>(rd, tab, lo, pos, ns, A);
    transpose_planes(A);
#pragma unroll
    for (int s = 0; s < 16; ++s)
        cf[order_of(s)] = A[s] - kNega;
    return nz;
}

// A lane's view of the code from the group starting at bit `start`.
__device__ __forceinline__ void lane_view(const uint32_t* code, uint64_t nwords, uint64_t start, const uint32_t*& g,
                                          uint32_t& lim, uint32_t& pos)
{
    const uint64_t q = start >> 5;
    const uint64_t left = q < nwords ? nwords - q : 0;
    g = code + (q < nwords ? q : 0);
    lim = (uint32_t)(left < 0xFFFFFFFFull ? left : 0xFFFFFFFFull);
    pos = (uint32_t)(start & 31u);
}

// A lane's ring: `head` is the view word (counted from the 16-byte boundary
// at or before the view's first word) up to which it is filled, a multiple
// of 4; `hs` the ring piece (0..5) that word goes to.  Both start at 0.
struct VarRing {
    uint32_t head = 0u, hs = 0u;
};

// The next block of a lane's view at bit pos (advanced past it): the ring is
// refilled through 24 words from the block's 16-byte piece and the block
// decoded there.  A piece inside the view is one 16-byte load, a piece
// reaching before the view's first word or past its end is read word by word
// (zero outside).  A block that read past the ring would be decoded again
// from global memory; by the bound above that never happens for codes of at
// most 32 planes, and the check keeps a code that breaks the bound (a
// corrupt stream) from decoding out of stale ring words.
template <int T>
__device__ __forceinline__ bool var_next_block(const uint32_t* g, uint32_t lim, uint32_t* row, const uint32_t* tab,
                                               int mode, int param, bool live, uint32_t& pos, int& emax,
                                               uint32_t (&cf)[16], VarRing& ring)
{
    constexpr uint32_t kPieces = kVarRing / 4;
    const uint32_t a = (uint32_t)(reinterpret_cast<uintptr_t>(g) >> 2) & 3u; // g's word within its 16 bytes
    const uint32_t b = ((pos >> 5) + a) & ~3u; // the block's first piece, in words from g - a
    const uint32_t h0 = __builtin_elementwise_max(ring.head, b);
    const uint32_t n = live ? (b + kVarRing - h0) >> 2 : 0u; // pieces to load
    u32x4 v[kPieces];
#pragma unroll
    for (uint32_t k = 0; k < kPieces; ++k) {
        v[k] = u32x4{0u, 0u, 0u, 0u};
        if (__any(k < n)) {
            if (k < n) {
                const int64_t s0 = (int64_t)(h0 + 4 * k) - (int64_t)a; // view word of the piece's first word
                if (s0 >= 0 && s0 + 4 <= (int64_t)lim) {
                    v[k] = *reinterpret_cast<const u32x4*>(g + s0);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        v[k][i] = (s0 + i >= 0 && s0 + i < (int64_t)lim) ? g[s0 + i] : 0u;
                }
            }
        }
    }
    // the pieces into their ring slots, piece h0 / 4 + k at slot c0 + k
    // (mod 6): on from the head's slot, or from slot 0 when the block starts
    // past the ring's end (all 6 pieces are new then)
    const uint32_t c0 = h0 > ring.head ? 0u : ring.hs;
#pragma unroll
    for (uint32_t k = 0; k < kPieces; ++k) {
        if (k < n) {
            uint32_t c = c0 + k;
            c = __builtin_elementwise_min(c, c - kPieces);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                row[(4 * c + i) * T] = v[k][i];
            if (c == 0)
                row[kVarRing * T] = v[k][0]; // the mirror word
        }
    }
    if (live) {
        const uint32_t hs = c0 + n;
        ring.hs = __builtin_elementwise_min(hs, hs - kPieces);
        ring.head = b + kVarRing;
    }
    // the block's piece b sits where the ring's head is now (24 words on)
    uint32_t lpos = pos + 32u * a - 32u * b;
    bool nz = var_block_coeffs(StagedBits<T>{row, 4u * ring.hs}, tab, mode, param, live, lpos, emax, cf);
    const bool over = live && lpos >= 32u * (kVarRing - 1u);
    if (__any(over)) {
        if (over) {
            uint32_t p = pos;
            nz = var_block_coeffs(GlobalBits{g, lim}, tab, mode, param, true, p, emax, cf);
            lpos = p + 32u * a - 32u * b;
        }
    }
    pos = lpos + 32u * b - 32u * a;
    return nz;
}

// Whole matrix into row-major FP32: one lane per (block row, group), in
// 256-lane workgroups.  A lane holds kVarSpan decoded blocks in registers
// (134 VGPRs, within the two waves per SIMD that LDS allows) and then
// writes each of its 4 rows as kVarSpan adjacent 16-byte stores, 64
// contiguous bytes.  The stores are ordinary (cached) ones, so that L2 can
// gather a lane's pieces of a row into whole lines: non-temporal stores of
// single blocks, from lanes 512 bytes apart, took 2.6 times as long at
// 8192^2.
constexpr int kVarSpan = 4;

__global__ void __launch_bounds__(kVarThreadsSmall) var_decode_kernel(
    const uint64_t* __restrict__ index, const uint32_t* __restrict__ code, uint64_t nwords, int mode, int param,
    uint32_t rows, uint32_t cols, uint32_t nbc, uint32_t ngroups, uint64_t nlanes, float* __restrict__ out)
{
    constexpr int T = kVarThreadsSmall;
    static_assert(32 % kVarSpan == 0, "spans tile a group");
    __shared__ uint32_t tab[kSecEntries];
    __shared__ uint32_t stage[T * kVarRow];
    uint32_t* row = stage + threadIdx.x;
    load_table<T>(tab);
    const uint64_t lane_id = (uint64_t)blockIdx.x * T + threadIdx.x;
    const bool in = lane_id < nlanes;
    const uint32_t bi = in ? (uint32_t)(lane_id / ngroups) : 0u, a = in ? (uint32_t)(lane_id % ngroups) : 0u;
    const uint32_t* g;
    uint32_t lim, pos;
    lane_view(code, nwords, in ? index[lane_id] : 0ull, g, lim, pos);
    VarRing ring;
    // rows of whole blocks: every span of whole blocks starts 16-byte aligned
    const bool whole = (cols & 3u) == 0u;
    for (uint32_t j0 = 0; j0 < 32u; j0 += kVarSpan) {
        float v[kVarSpan][16];
#pragma unroll kVarSpan
        for (int s = 0; s < kVarSpan; ++s) {
            const uint32_t bj = a * 32u + j0 + s;
            int emax;
            uint32_t iv[16];
            var_next_block<T>(g, lim, row, tab, mode, param, in && bj < nbc, pos, emax, iv, ring);
            inv_xform(iv);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                v[s][i] = __builtin_ldexpf((float)(int32_t)iv[i], emax - 30);
        }
        const uint32_t bj0 = a * 32u + j0;
        if (!in || bj0 >= nbc)
            continue;
        if (whole && bj0 + kVarSpan <= nbc) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (4 * bi + r >= rows)
                    continue;
                f32x4* o = reinterpret_cast<f32x4*>(out + (uint64_t)(4 * bi + r) * cols + 4 * bj0);
#pragma unroll
                for (int s = 0; s < kVarSpan; ++s)
                    o[s] = f32x4{v[s][4 * r], v[s][4 * r + 1], v[s][4 * r + 2], v[s][4 * r + 3]};
            }
        } else {
            // the matrix edge: value by value
#pragma unroll
            for (int s = 0; s < kVarSpan; ++s) {
                const uint32_t bj = bj0 + s;
                if (bj >= nbc)
                    continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * bi + r >= rows)
                        continue;
                    float* o = out + (uint64_t)(4 * bi + r) * cols + 4 * bj;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (4 * bj + c < cols)
                            o[c] = v[s][4 * r + c];
                }
            }
        }
    }
}

struct VarFp64Acc {
    double s;
    __device__ __forceinline__ void zero() { s = 0.0; }
    __device__ __forceinline__ void add(float p) { s += (double)p; }
    __device__ __forceinline__ double value() const { return s; }
    __device__ __forceinline__ void merge_from_lane(int mask) { s += __shfl_xor(s, mask, 64); }
};

struct VarTwoSumAcc {
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

// Fused decode + GEMV over block rows [bi_begin, bi_end): G = 2^lg lanes
// (1..8) per block row, T / G block rows per workgroup; lane gl of a row
// takes group slab * G + gl (32 blocks).  Output row i of the range is
// matrix row 4 * bi_begin + skip + i.
template <int T, typename Acc>
__global__ void __launch_bounds__(T) var_gemv_kernel(
    const uint64_t* __restrict__ index, const uint32_t* __restrict__ code, uint64_t nwords, int mode, int param,
    const float* __restrict__ u, float* __restrict__ y, double* __restrict__ part, uint32_t nbc, uint32_t ngroups,
    uint32_t bi_begin, uint32_t bi_end, uint32_t nslab, uint32_t cols, uint32_t nrows, uint32_t skip, uint32_t lg)
{
    __shared__ uint32_t tab[kSecEntries];
    // the lanes' staging rows; after the blocks, the row sums per group
    // (<= 512) and row of the block
    __shared__ double stage_d[T * kVarRow / 2];
    static_assert(kVarRow * T / 2 >= 4 * T, "the row sums fit the staging area");
    uint32_t* row = reinterpret_cast<uint32_t*>(stage_d) + threadIdx.x;
    double* red = stage_d;
    load_table<T>(tab);
    const uint32_t G = 1u << lg, groups = (uint32_t)T >> lg;
    const uint32_t grp = threadIdx.x >> lg, gl = threadIdx.x & (G - 1);
    const uint32_t tile = blockIdx.x / nslab, slab = blockIdx.x % nslab;
    const uint32_t bi = bi_begin + tile * groups + grp;
    const uint32_t a = slab * G + gl;
    const bool in = bi < bi_end && a < ngroups;
    const uint32_t* g;
    uint32_t lim, pos;
    lane_view(code, nwords, in ? index[(uint64_t)bi * ngroups + a] : 0ull, g, lim, pos);
    VarRing ring;
    Acc acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        acc[r].zero();
    for (uint32_t j = 0; j < 32u; ++j) {
        const uint32_t bj = a * 32u + j;
        const bool live = in && bj < nbc;
        float uu[4] = {0.f, 0.f, 0.f, 0.f};
        if (live) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                uu[c] = 4 * bj + c < cols ? u[4 * bj + c] : 0.0f;
        }
        int emax;
        uint32_t iv[16];
        const bool nz = var_next_block<T>(g, lim, row, tab, mode, param, live, pos, emax, iv, ring);
        if (live && nz) {
            // the exact integer inverse transform (not B (C (B^T u))): a
            // coefficient cut to its top planes can reach -2^31, where the
            // lift wraps modulo 2^32 as the decoded matrix does
            inv_xform(iv);
            const int k = emax - 30;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = (float)(int32_t)iv[4 * r] * uu[0];
                v = __builtin_fmaf((float)(int32_t)iv[4 * r + 1], uu[1], v);
                v = __builtin_fmaf((float)(int32_t)iv[4 * r + 2], uu[2], v);
                v = __builtin_fmaf((float)(int32_t)iv[4 * r + 3], uu[3], v);
                acc[r].add(__builtin_ldexpf(v, k));
            }
        }
    }
    // across the G lanes of the row (within a wave), then one lane per row;
    // the row sums reuse the staging area once every lane is done with it
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        for (int mask = (int)G >> 1; mask >= 1; mask >>= 1)
            acc[r].merge_from_lane(mask);
        if (gl == 0)
            red[grp * 4 + r] = acc[r].value();
    }
    __syncthreads();
    if (threadIdx.x >= groups)
        return;
    const uint32_t row_bi = bi_begin + tile * groups + threadIdx.x;
    if (row_bi >= bi_end)
        return;
    double v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        v[r] = red[threadIdx.x * 4 + r];
    const uint32_t part_rows = (bi_end - bi_begin) * 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint32_t local = (row_bi - bi_begin) * 4 + r;
        if (nslab > 1)
            part[(uint64_t)slab * part_rows + local] = v[r];
        else if (local >= skip && local - skip < nrows)
            y[local - skip] = (float)v[r];
    }
}

// Slab partials [nslab][part_rows] -> y[0, nrows) (y[i] from row skip + i),
// one lane per row, slabs in order.
__global__ void __launch_bounds__(256) var_reduce_kernel(const double* __restrict__ part, uint32_t part_rows,
                                                         uint32_t skip, uint32_t nrows, uint32_t nslab,
                                                         float* __restrict__ y)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nrows; i += stride) {
        double s = 0.0;
        for (uint32_t q = 0; q < nslab; ++q)
            s += part[(uint64_t)q * part_rows + skip + i];
        y[i] = (float)s;
    }
}

unsigned grid_of(uint64_t items, unsigned threads)
{
    const uint64_t g = (items + threads - 1) / threads;
    return (unsigned)(g ? (g < (1u << 30) ? g : (1u << 30)) : 1);
}

// ------------------------------------------------------------ host encoder
// The same code, written on the host (bit s of the stream is bit s % 8 of
// byte s / 8).
struct HostBits {
    std::vector<uint64_t> w;
    uint64_t pos = 0;
    void put(uint32_t bit)
    {
        if ((pos >> 6) >= w.size())
            w.push_back(0);
        if (bit & 1u)
            w[pos >> 6] |= 1ull << (pos & 63u);
        ++pos;
    }
};

int32_t h_asr1(int32_t v) { return v >> 1; }

// forward lift on p[0], p[s], p[2s], p[3s] (modulo 2^32, floor halving)
void h_fwd_lift(uint32_t* p, int s)
{
    uint32_t x = p[0], y = p[s], z = p[2 * s], w = p[3 * s];
    x = (uint32_t)h_asr1((int32_t)(x + w));
    w -= x;
    z = (uint32_t)h_asr1((int32_t)(z + y));
    y -= z;
    x = (uint32_t)h_asr1((int32_t)(x + z));
    z -= x;
    w = (uint32_t)h_asr1((int32_t)(w + y));
    y -= w;
    w += (uint32_t)h_asr1((int32_t)y);
    y -= (uint32_t)h_asr1((int32_t)w);
    p[0] = x;
    p[s] = y;
    p[2 * s] = z;
    p[3 * s] = w;
}

int h_binade(float f)
{
    int e;
    frexpf(f, &e);
    return e;
}

// One block (f: local index 4r + c).  Returns false for NaN/Inf.
bool h_encode_block(HostBits& b, const float f[16], int mode, int param)
{
    static constexpr int kOrder[16] = {0, 1, 4, 5, 2, 8, 6, 9, 3, 12, 10, 7, 13, 11, 14, 15};
    bool nonzero = false;
    int emax = -126;
    for (int v = 0; v < 16; ++v) {
        if (!(f[v] == f[v]) || f[v] - f[v] != 0.0f)
            return false;
        if (f[v] != 0.0f) {
            const int e = h_binade(f[v]);
            emax = nonzero ? std::max(emax, e) : e;
            nonzero = true;
        }
    }
    if (!nonzero) {
        b.put(0);
        return true;
    }
    emax = std::max(emax, -126);
    b.put(1);
    for (int k = 0; k < 8; ++k)
        b.put(((uint32_t)(emax + 127) >> k) & 1u);
    uint32_t iv[16];
    for (int v = 0; v < 16; ++v)
        iv[v] = (uint32_t)(int32_t)std::trunc(std::ldexp((double)f[v], 30 - emax));
    for (int r = 0; r < 4; ++r)
        h_fwd_lift(iv + 4 * r, 1);
    for (int c = 0; c < 4; ++c)
        h_fwd_lift(iv + c, 4);
    uint32_t n[16];
    for (int s = 0; s < 16; ++s)
        n[s] = (iv[kOrder[s]] + 0xAAAAAAAAu) ^ 0xAAAAAAAAu;
    const int lo = 32 - var_planes(mode, param, emax);
    uint32_t nsig = 0;
    for (int p = 31; p >= lo; --p) {
        uint32_t x = 0;
        for (int s = 0; s < 16; ++s)
            x |= ((n[s] >> p) & 1u) << s;
        for (uint32_t k = 0; k < nsig; ++k)
            b.put((x >> k) & 1u);
        x >>= nsig;
        while (nsig < 16) {
            const uint32_t grp = x != 0;
            b.put(grp);
            if (!grp)
                break;
            while (nsig < 15) {
                const uint32_t bit = x & 1u;
                b.put(bit);
                if (bit)
                    break;
                x >>= 1;
                ++nsig;
            }
            x >>= 1;
            ++nsig;
        }
    }
    return true;
}

} // namespace

uint32_t var_groups(uint32_t cols) { return (((cols + 3) / 4) + 31) / 32; }
uint64_t var_index_bytes(uint32_t rows, uint32_t cols) { return (uint64_t)((rows + 3) / 4) * var_groups(cols) * 8; }

bool var_mode(int fmt, uint32_t rate, int& mode, int& param)
{
    if (fmt == WH_FMT_ZFP_FIXED_PRECISION && rate >= 1 && rate <= 32) {
        mode = 0;
        param = (int)rate;
        return true;
    }
    if (fmt == WH_FMT_ZFP_FIXED_ACCURACY && rate >= 1024 - 160 && rate <= 1024 + 160) {
        mode = 1;
        param = (int)rate - 1024;
        return true;
    }
    return false;
}

hipError_t var_decode(const Matrix& m, float* out, hipStream_t st)
{
    int mode, param;
    if (!var_mode(m.desc.fmt, m.desc.rate, mode, param))
        return hipErrorInvalidValue;
    const uint32_t nbc = (m.desc.cols + 3) / 4, ng = var_groups(m.desc.cols);
    const uint64_t nlanes = (uint64_t)((m.desc.rows + 3) / 4) * ng;
    const uint64_t ib = var_index_bytes(m.desc.rows, m.desc.cols);
    const uint64_t* index = static_cast<const uint64_t*>(m.dptr);
    const uint32_t* code = reinterpret_cast<const uint32_t*>(static_cast<const char*>(m.dptr) + ib);
    const uint64_t nwords = (m.nbytes - ib) / 4;
    hipLaunchKernelGGL(var_decode_kernel, dim3(grid_of(nlanes, kVarThreadsSmall)), dim3(kVarThreadsSmall), 0, st,
                       index, code, nwords, mode, param, m.desc.rows, m.desc.cols, nbc, ng, nlanes, out);
    return hipGetLastError();
}

// Launch shape: G lanes per block row, the smallest power of two (1..8)
// that covers the row's groups, or 8; slabs of G groups; workgroups of
// `threads` lanes.
struct VarPlan {
    uint32_t lg, nslab, ntiles, bi_begin, bi_end, threads;
};

VarPlan var_plan(const Matrix& m, uint32_t row_begin, uint32_t row_end)
{
    VarPlan p{};
    const uint32_t ng = var_groups(m.desc.cols);
    p.lg = 0;
    while (p.lg < 3 && (1u << p.lg) < ng)
        ++p.lg;
    p.nslab = (ng + (1u << p.lg) - 1) >> p.lg;
    p.bi_begin = row_begin / 4;
    p.bi_end = (row_end + 3) / 4;
    const uint64_t lanes = (uint64_t)(p.bi_end - p.bi_begin) * p.nslab << p.lg;
    p.threads = lanes >= kVarLargeFrom ? kVarThreadsLarge : kVarThreadsSmall;
    const uint32_t rows_per_tile = p.threads >> p.lg;
    p.ntiles = (p.bi_end - p.bi_begin + rows_per_tile - 1) / rows_per_tile;
    return p;
}

size_t var_partials(const Matrix& m, uint32_t row_begin, uint32_t row_end)
{
    const VarPlan p = var_plan(m, row_begin, row_end);
    return p.nslab > 1 ? (size_t)p.nslab * (p.bi_end - p.bi_begin) * 4 : 0;
}

hipError_t var_gemv(const Matrix& m, AccMode acc, const float* u, float* y, uint32_t row_begin, uint32_t row_end,
                    double* part, hipStream_t st)
{
    int mode, param;
    if (!var_mode(m.desc.fmt, m.desc.rate, mode, param))
        return hipErrorInvalidValue;
    const VarPlan p = var_plan(m, row_begin, row_end);
    if (p.ntiles == 0)
        return hipSuccess;
    const uint32_t nbc = (m.desc.cols + 3) / 4, ng = var_groups(m.desc.cols);
    const uint64_t ib = var_index_bytes(m.desc.rows, m.desc.cols);
    const uint64_t* index = static_cast<const uint64_t*>(m.dptr);
    const uint32_t* code = reinterpret_cast<const uint32_t*>(static_cast<const char*>(m.dptr) + ib);
    const uint64_t nwords = (m.nbytes - ib) / 4;
    const uint32_t nrows = row_end - row_begin, skip = row_begin & 3u;
    const dim3 grid(p.ntiles * p.nslab);
    const dim3 block(p.threads);
    if (acc == AccMode::TwoSum && p.threads == kVarThreadsLarge)
        hipLaunchKernelGGL((var_gemv_kernel<kVarThreadsLarge, VarTwoSumAcc>), grid, block, 0, st, index, code, nwords,
                           mode, param, u, y, part, nbc, ng, p.bi_begin, p.bi_end, p.nslab, m.desc.cols, nrows, skip,
                           p.lg);
    else if (acc == AccMode::TwoSum)
        hipLaunchKernelGGL((var_gemv_kernel<kVarThreadsSmall, VarTwoSumAcc>), grid, block, 0, st, index, code, nwords,
                           mode, param, u, y, part, nbc, ng, p.bi_begin, p.bi_end, p.nslab, m.desc.cols, nrows, skip,
                           p.lg);
    else if (p.threads == kVarThreadsLarge)
        hipLaunchKernelGGL((var_gemv_kernel<kVarThreadsLarge, VarFp64Acc>), grid, block, 0, st, index, code, nwords,
                           mode, param, u, y, part, nbc, ng, p.bi_begin, p.bi_end, p.nslab, m.desc.cols, nrows, skip,
                           p.lg);
    else
        hipLaunchKernelGGL((var_gemv_kernel<kVarThreadsSmall, VarFp64Acc>), grid, block, 0, st, index, code, nwords,
                           mode, param, u, y, part, nbc, ng, p.bi_begin, p.bi_end, p.nslab, m.desc.cols, nrows, skip,
                           p.lg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.nslab == 1)
        return e;
    hipLaunchKernelGGL(var_reduce_kernel, dim3(grid_of(nrows, 256)), dim3(256), 0, st, part,
                       (p.bi_end - p.bi_begin) * 4, skip, nrows, p.nslab, y);
    return hipGetLastError();
}

} // namespace wh

using namespace wh;

extern "C" uint64_t wh_var_index_bytes(uint32_t rows, uint32_t cols) { return var_index_bytes(rows, cols); }

extern "C" uint64_t wh_var_capacity_bytes(uint32_t rows, uint32_t cols)
{
    // header + 32 planes of at most 16 verbatim and 17 section bits each
    return var_index_bytes(rows, cols) + (uint64_t)((rows + 3) / 4) * ((cols + 3) / 4) * ((9 + 32 * 33 + 7) / 8) + 24;
}

extern "C" wh_status wh_encode_var(const float* h_M, uint32_t rows, uint32_t cols, int32_t fmt, uint32_t rate,
                                   void* h_out, uint64_t cap, uint64_t* out_bytes)
{
    int mode, param;
    if (!h_M || !h_out || !out_bytes)
        return WH_ERR_INVALID;
    if (rows == 0 || cols == 0)
        return WH_ERR_SHAPE;
    if (!var_mode(fmt, rate, mode, param))
        return WH_ERR_FORMAT;
    try {
        const uint32_t nbr = (rows + 3) / 4, nbc = (cols + 3) / 4, ng = var_groups(cols);
        const uint64_t ib = var_index_bytes(rows, cols);
        if (cap < ib + 16)
            return WH_ERR_INVALID;
        // block rows encoded in parallel, each into its own bit buffer
        std::vector<HostBits> rowbits(nbr);
        std::vector<std::vector<uint64_t>> rowidx(nbr, std::vector<uint64_t>(ng));
        std::vector<char> bad(nbr, 0);
        const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nth; ++t)
            th.emplace_back([&, t] {
                for (uint32_t bi = t; bi < nbr; bi += nth) {
                    HostBits& b = rowbits[bi];
                    for (uint32_t bj = 0; bj < nbc; ++bj) {
                        if (bj % 32 == 0)
                            rowidx[bi][bj / 32] = b.pos;
                        float f[16];
                        for (int r = 0; r < 4; ++r)
                            for (int c = 0; c < 4; ++c) {
                                const uint32_t i = std::min(4 * bi + r, rows - 1), j = std::min(4 * bj + c, cols - 1);
                                f[4 * r + c] = h_M[(uint64_t)i * cols + j];
                            }
                        if (!h_encode_block(b, f, mode, param))
                            bad[bi] = 1;
                    }
                }
            });
        for (auto& x : th)
            x.join();
        if (std::find(bad.begin(), bad.end(), 1) != bad.end())
            return WH_ERR_INVALID;
        uint64_t total = 0;
        for (uint32_t bi = 0; bi < nbr; ++bi)
            total += rowbits[bi].pos;
        // 16 zero bytes of reader padding, whole 8-byte words
        const uint64_t code_bytes = ((total + 7) / 8 + 16 + 7) / 8 * 8;
        if (ib + code_bytes > cap)
            return WH_ERR_INVALID;
        char* out = static_cast<char*>(h_out);
        memset(out, 0, (size_t)(ib + code_bytes));
        uint64_t* index = reinterpret_cast<uint64_t*>(out);
        uint8_t* code = reinterpret_cast<uint8_t*>(out + ib);
        uint64_t off = 0;
        for (uint32_t bi = 0; bi < nbr; ++bi) {
            for (uint32_t a = 0; a < ng; ++a)
                index[(uint64_t)bi * ng + a] = off + rowidx[bi][a];
            const HostBits& b = rowbits[bi];
            for (uint64_t s = 0; s < b.pos; s += 64) { // splice the row's bits at off
                const uint32_t n = (uint32_t)std::min<uint64_t>(64, b.pos - s);
                const uint64_t v = b.w[s >> 6];
                for (uint32_t k = 0; k < n; k += 8) {
                    const uint64_t at = off + s + k;
                    const uint32_t nb = std::min(8u, n - k);
                    const uint32_t byte = (uint32_t)(v >> k) & ((1u << nb) - 1u);
                    code[at >> 3] |= (uint8_t)(byte << (at & 7u));
                    if ((at & 7u) + nb > 8)
                        code[(at >> 3) + 1] |= (uint8_t)(byte >> (8u - (at & 7u)));
                }
            }
            off += b.pos;
        }
        *out_bytes = ib + code_bytes;
        return WH_OK;
    } catch (const std::bad_alloc&) {
        return WH_ERR_NOMEM;
    } catch (...) {
        return WH_ERR_INVALID;
    }
}
