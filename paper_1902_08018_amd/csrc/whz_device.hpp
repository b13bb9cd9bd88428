// whz_device.hpp -- WHZ1 block codec, device side (gfx950).
//
// WHZ1 is this library's zfp-style fixed-rate code for FP32 matrices in 4x4
// blocks (the paper stores its matrices zfp-compressed in fixed-rate mode,
// Sec. 4.3, Table 2).  Per block, exactly maxbits = 16*rate bits, LSB-first:
//   bit 0          1 if any value is nonzero (else the block is all +0)
//   bits 1..8      E = emax + 127, emax = max binade exponent, >= -126
//   bits 9..       embedded bit-plane code of the 16 transform coefficients,
//                  planes 31 -> 0, truncated at maxbits, zero padded.
// Coefficients: i = trunc(f * 2^(30 - emax)); a 4-point lift along every
// block row then every block column; sequency order; negabinary.
//
// One lane decodes one block.  The bits of the lane's block sit in a
// lane-private LDS row (words 0..NW-1 plus three zero words), so a 64-bit
// window can be read at any bit position with two funnel shifts.
//
// Included by the .hip translation units after <hip/hip_runtime.h>.
#pragma once

#include <stdint.h>

namespace wh {

constexpr uint32_t kNega = 0xAAAAAAAAu;

// Sequency order: coefficient number s of the code is the transform output
// at local index kOrder(s) = 4r + c (c: horizontal frequency, r: vertical).
// Ordered by c + r, then c^2 + r^2, then larger c first.
__device__ __forceinline__ constexpr int order_of(int s)
{
    constexpr int t[16] = {0, 1, 4, 5, 2, 8, 6, 9, 3, 12, 10, 7, 13, 11, 14, 15};
    return t[s];
}

// ((hi:lo) >> sh) & 0xffffffff for sh in [0, 31]
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

// The word of a staged row that holds bit position pos: pos >> 5.  On the
// GPU the shift is opaque to the compiler, so a row address q * STRIDE +
// base stays one shift-add; seen through, (pos >> 5) << 11 is rewritten as
// a shift and a mask, one instruction more per window read.  The host build
// of this header (CPU tests) takes the plain shift.
__device__ __forceinline__ uint32_t word_of(uint32_t pos)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t q;
    asm("v_lshrrev_b32 %0, 5, %1" : "=v"(q) : "v"(pos));
    return q;
#else
    return pos >> 5;
#endif
}

__device__ __forceinline__ uint32_t asr1(uint32_t v) { return (uint32_t)((int32_t)v >> 1); }

// ---------------------------------------------------------------- lifting
// Forward lift on (x, y, z, w), modulo 2^32, floor halving.
__device__ __forceinline__ void fwd_lift(uint32_t& x, uint32_t& y, uint32_t& z, uint32_t& w)
{
    x = asr1(x + w);
    w -= x;
    z = asr1(z + y);
    y -= z;
    x = asr1(x + z);
    z -= x;
    w = asr1(w + y);
    y -= w;
    w += asr1(y);
    y -= asr1(w);
}

// Inverse lift.  Each "a <- a + b; b <- 2b - a" pair is written in its
// equivalent form "a' = a + b; b' = b - a" (both modulo 2^32).
__device__ __forceinline__ void inv_lift(uint32_t& x, uint32_t& y, uint32_t& z, uint32_t& w)
{
    y += asr1(w);
    w -= asr1(y);
    uint32_t t = y;
    y += w;
    w -= t;
    t = z;
    z += x;
    x -= t;
    t = y;
    y += z;
    z -= t;
    t = w;
    w += x;
    x -= t;
}

// 2-D inverse transform, local index v = 4r + c: columns, then rows.
__device__ __forceinline__ void inv_xform(uint32_t (&v)[16])
{
#pragma unroll
    for (int c = 0; c < 4; ++c)
        inv_lift(v[c], v[c + 4], v[c + 8], v[c + 12]);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        inv_lift(v[4 * r], v[4 * r + 1], v[4 * r + 2], v[4 * r + 3]);
}

__device__ __forceinline__ void fwd_xform(uint32_t (&v)[16])
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
        fwd_lift(v[4 * r], v[4 * r + 1], v[4 * r + 2], v[4 * r + 3]);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        fwd_lift(v[c], v[c + 4], v[c + 8], v[c + 12]);
}

// ------------------------------------------------------ bit-matrix transpose
// A[q] holds plane q in bits 0..15 and plane q+16 in bits 16..31 (bit s of a
// plane = coefficient s).  Afterwards A[s] is coefficient s: bit p = its bit
// in plane p.  Both 16x16 halves are transposed at once (the masks repeat in
// each 16-bit half, and every shifted bit that crosses a half is masked off).
// One stage: rows i and i + D (i & D == 0) exchange their D-wide column
// blocks; M selects the low D columns of every 2D-wide group.  Templates keep
// every index a compile-time constant (no register indexing, no loop).
template <int D, uint32_t M, int I>
__device__ __forceinline__ void transpose_pairs(uint32_t (&A)[16])
{
    if constexpr (I < 16) {
        if constexpr ((I & D) == 0) {
            const uint32_t a = A[I], b = A[I + D];
            A[I] = (a & M) | ((b << D) & ~M);
            A[I + D] = ((a >> D) & M) | (b & ~M);
        }
        transpose_pairs<D, M, I + 1>(A);
    }
}

// The first stage (8-wide blocks) moves whole bytes: each output register
// takes two bytes from each input, one byte permute per register.
template <int I>
__device__ __forceinline__ void transpose_bytes(uint32_t (&A)[16])
{
    if constexpr (I < 8) {
        const uint32_t a = A[I], b = A[I + 8];
        // selector bytes index (a: 0..3, b: 4..7), low output byte first
        A[I] = __builtin_amdgcn_perm(b, a, 0x06020400u);     // a.b0 b.b0 a.b2 b.b2
        A[I + 8] = __builtin_amdgcn_perm(b, a, 0x07030501u); // a.b1 b.b1 a.b3 b.b3
        transpose_bytes<I + 1>(A);
    }
}

__device__ __forceinline__ void transpose_planes(uint32_t (&A)[16])
{
    transpose_bytes<0>(A);
    transpose_pairs<4, 0x0F0F0F0Fu, 0>(A);
    transpose_pairs<2, 0x33333333u, 0>(A);
    transpose_pairs<1, 0x55555555u, 0>(A);
}

// --------------------------------------------------------------- decoding
// Group-test sections are decoded with a lookup table of 8 stream bits at a
// time.  A section (after the verbatim bits of a plane) is a sequence of
// tokens: "0" (next coefficient stays insignificant), "11" (it becomes
// significant, another group follows), "10" (it becomes significant, the
// plane ends); a group bit 0 at the start ends the plane at once, and when
// the scan reaches coefficient 15 inside a run its 1 is implied.
//
// Table entry for (nsig, state, 8 bits), state 0 = at a group bit, 1 =
// inside a run; index nsig * kSecRow + (state << 8) + bits.  The row stride
// kSecRow = 513 is odd on purpose: the decoder carries ns = nsig * kSecRow
// instead of nsig, and since 513 = 16 * 32 + 1, ns's low byte (and its low
// five bits, all that v_bfe reads of an offset or a width) is nsig itself.
// The first lookup's address is then one add of ns and the 8 bits.  The
// fields sit where the decoder can take them without masking:
//   bits  0..15  coefficients that became significant, at their absolute
//                positions (the table is indexed by nsig), including
//                coefficient 15's implied 1; they OR straight into the plane
//                word's low half
//   bits 16..19  stream bits consumed (0..8); bits 20..23 are zero, so the
//                whole byte is the count
//   bit  24      state to continue in when the section did not end
//   bits 25..28  coefficients passed (nsig advances by this much, 0..9)
//   bit  31      the section ended: the sign bit, tested without a mask
// (e >> 16) & 0x8100 puts the state at index bit 8 and the ended flag at bit
// 15, past every index of the table.  One more entry, kSecDone, is "ended,
// nothing consumed": a lane whose section has ended reads it, so every step
// runs unpredicated.
constexpr int kSecBits = 8;
constexpr int kSecN = 17; // nsig 0..16
constexpr int kSecRow = 2 * (1 << kSecBits) + 1;
constexpr int kSecDone = kSecN * kSecRow;
constexpr int kSecEntries = kSecDone + 1;
constexpr uint32_t kEntState = 1u << 24, kEntDone = 1u << 31;
static_assert(kSecDone <= (int)(kEntDone >> 16), "the done flag must lift an index past the table");
static_assert((kSecRow & 0x1FF) == 1 && (kSecN - 1) * kSecRow + 2 * (1 << kSecBits) <= kSecDone,
              "ns = nsig * kSecRow keeps nsig in its low byte, and rows do not overlap");
// nsig from ns = nsig * kSecRow (nsig <= 16)
__host__ __device__ __forceinline__ constexpr uint32_t ns_nsig(uint32_t ns) { return ns & 0xFFu; }

// a + nsig for ns = nsig * kSecRow.  On the GPU one SDWA add reads ns's low
// byte; written plainly the compiler masks first and adds in a second
// instruction.
__device__ __forceinline__ uint32_t add_nsig(uint32_t a, uint32_t ns)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:DWORD"
        : "=v"(r)
        : "v"(ns), "v"(a));
    return r;
#else
    return a + ns_nsig(ns);
#endif
}

// tab[ns + bits] (tab in LDS).  On the GPU the byte address is one
// v_add_lshl; written plainly the compiler scales both terms apart.
__device__ __forceinline__ uint32_t sec_lookup(const uint32_t* tab, uint32_t ns, uint32_t bits)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t off;
    asm("v_add_lshl_u32 %0, %1, %2, 2" : "=v"(off) : "v"(ns), "v"(bits));
    return *(const uint32_t*)((const char*)tab + off);
#else
    return tab[ns + bits];
#endif
}

// a + (b & 0xFF).  On the GPU one SDWA add reads b's low byte.
__device__ __forceinline__ uint32_t add_byte0(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:DWORD"
        : "=v"(r)
        : "v"(b), "v"(a));
    return r;
#else
    return a + (b & 0xFFu);
#endif
}

// tab[min(i + j, kSecDone)] (tab in LDS).  On the GPU the byte offset is one
// v_add_lshl and the clamp one v_min on it; written plainly the compiler adds,
// clamps and then scales.
__device__ __forceinline__ uint32_t sec_lookup_clamped(const uint32_t* tab, uint32_t i, uint32_t j)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t off;
    asm("v_add_lshl_u32 %0, %1, %2, 2" : "=v"(off) : "v"(i), "v"(j));
    off = __builtin_elementwise_min(off, 4u * (uint32_t)kSecDone);
    return *(const uint32_t*)((const char*)tab + off);
#else
    return tab[__builtin_elementwise_min(i + j, (uint32_t)kSecDone)];
#endif
}

__host__ __device__ __forceinline__ constexpr uint32_t ent_used(uint32_t e) { return (e >> 16) & 0xFFu; }
__host__ __device__ __forceinline__ constexpr uint32_t ent_adv(uint32_t e) { return (e >> 25) & 15u; }
__host__ __device__ __forceinline__ constexpr bool ent_open(uint32_t e) { return (int32_t)e >= 0; }
// the entry's part of the next index: state at bit 8, ended flag at bit 15
__host__ __device__ __forceinline__ constexpr uint32_t ent_next(uint32_t e) { return (e >> 16) & 0x8100u; }

__host__ __device__ constexpr uint32_t section_entry(int state, int nsig, int bits)
{
    int used = 0, adv = 0, done = 0, st = state;
    uint32_t ones = 0;
    for (;;) {
        if (st == 0) {
            if (nsig + adv >= 16) { // every coefficient significant: no group bit
                done = 1;
                break;
            }
            if (used == kSecBits)
                break;
            const int g = (bits >> used) & 1;
            ++used;
            if (!g) {
                done = 1;
                break;
            }
            st = 1;
        } else {
            if (nsig + adv == 15) { // coefficient 15: its 1 is implied, not read
                ones |= 1u << 15;
                ++adv;
                done = 1;
                break;
            }
            if (used == kSecBits)
                break;
            const int b = (bits >> used) & 1;
            ++used;
            if (b) {
                ones |= 1u << (nsig + adv);
                st = 0;
            }
            ++adv;
        }
    }
    return ones | (uint32_t)used << 16 | (done ? 0u : (uint32_t)st << 24) | (uint32_t)adv << 25 |
           (done ? kEntDone : 0u);
}

struct SectionTable {
    uint32_t e[kSecEntries];
    constexpr SectionTable() : e()
    {
        for (int n = 0; n < kSecN; ++n)
            for (int st = 0; st < 2; ++st)
                for (int b = 0; b < (1 << kSecBits); ++b)
                    e[n * kSecRow + (st << 8) + b] = section_entry(st, n, b);
        e[kSecDone] = kEntDone;
    }
};

// A[q] starts as plane q | plane q+16 << 16 with every odd plane
// complemented: the transpose then yields n ^ 0xAAAAAAAA for each negabinary
// coefficient n, the first half of the conversion to two's complement.  (The
// variable-rate decoder keeps this form; the fixed-rate one stores the planes
// as they are and converts after the transpose.)
__host__ __device__ constexpr uint32_t kOddPlanes(int q) { return (q & 1) ? 0xFFFFFFFFu : 0u; }

// Negabinary n -> two's complement (n ^ 0xAAAAAAAA) - 0xAAAAAAAA, modulo
// 2^32: one v_xad on the GPU.
__device__ __forceinline__ uint32_t nega_to_int(uint32_t n)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    // one SGPR operand at most (constant bus): the addend comes in a VGPR
    asm("v_xad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(n), "s"(kNega), "v"(0u - kNega));
    return r;
#else
    return (n ^ kNega) - kNega;
#endif
}

// Plane P's word, (acc & 0xFFFF) | xv (disjoint bits), into A: plane P >= 16
// as the high half of A[P - 16] (low half zero); plane P < 16 as the low half
// of A[P], whose high half already holds plane P + 16.  One instruction each:
// an SDWA or writing one half of its destination (the other half zeroed, or
// kept).
template <int P>
__device__ __forceinline__ void store_plane(uint32_t (&A)[16], uint32_t acc, uint32_t xv)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (P >= 16)
        asm("v_or_b32_sdwa %0, %1, %2 dst_sel:WORD_1 dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:DWORD"
            : "=v"(A[P - 16])
            : "v"(acc), "v"(xv));
    else
        asm("v_or_b32_sdwa %0, %1, %2 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
            : "+v"(A[P])
            : "v"(acc), "v"(xv));
#else
    const uint32_t x = (acc & 0xFFFFu) | xv;
    if constexpr (P >= 16)
        A[P - 16] = x << 16;
    else
        A[P] = (A[P] & 0xFFFF0000u) | x;
#endif
}

// One bit plane of the embedded code (plane P, decoded in lockstep by all
// lanes of the wave; P is a template argument so A[] is indexed at compile
// time).  Every step is straight-line code for all lanes.  A lane whose budget
// is spent keeps stepping over zero bits: a zero group bit ends each section
// at once, so its plane words stay zero and its significance count is
// unchanged.
//
// Bits past the end of the block read as zero.  That gives the exact result
// everywhere except when the bit budget runs out inside a run: there the
// zero bits walk on to coefficient 15, where the code instead sets the
// coefficient the run had reached when the budget ended.  The number of
// zeros read past the end says which one that was.  Only planes in which
// some lane of the wave is past its budget pay for that correction.
//
// Returns the wave's mask of lanes past their budget.
template <int NW, int STRIDE, int P>
__device__ __forceinline__ uint64_t decode_plane(const uint32_t* lw, const uint32_t* tab, uint32_t& pos,
                                                 uint32_t& ns, uint32_t (&A)[16])
{
    constexpr uint32_t kMaxBits = 32u * NW;
    // word of pos (positions stay below 1024: kMaxBits + 32 + one plane)
    uint32_t q = word_of(pos);
    // 32 bits from pos: the verbatim bits (nsig <= 16) and the first 8
    // section bits always fit
    const uint32_t lo = funnel(lw[(q + 1) * STRIDE], lw[q * STRIDE], pos & 31u);
    // (i) verbatim bits of the significant coefficients (v_bfe takes the
    // width mod 32: nsig)
    const uint32_t xv = __builtin_amdgcn_ubfe(lo, 0u, ns);
    // (ii) group tests, 8 bits per table lookup.  acc's low half collects
    // the plane's new ones; its high half is the latest entry's fields, so
    // the loop carries no separate copy of the entry
    uint32_t acc = sec_lookup(tab, ns, __builtin_amdgcn_ubfe(lo, ns, 8u));
    uint32_t at = add_nsig(pos, ns) + ent_used(acc); // next unread bit
    ns += ent_adv(acc) * (uint32_t)kSecRow;
    if (__any(ent_open(acc))) {
        do {
            q = word_of(at);
            const uint32_t bits = funnel(lw[(q + 1) * STRIDE], lw[q * STRIDE], at & 31u);
            // ended: the index is past kSecDone and clamps onto it
            acc = (acc & 0xFFFFu) | sec_lookup_clamped(tab, add_byte0(ns, bits), ent_next(acc));
            at += ent_used(acc);
            ns += ent_adv(acc) * (uint32_t)kSecRow;
        } while (__any(ent_open(acc)));
    }
    const uint64_t past = __ballot(at >= kMaxBits);
    if (__builtin_expect(past != 0, 0)) { // a branch, not selects on every plane
        // the implied 1 of coefficient 15 moves back to where the run stood
        // when the budget ended (ex = zeros read past the end; ex <= 15
        // wherever that 1 is set)
        const uint32_t ex = __builtin_elementwise_sub_sat(at, kMaxBits);
        const uint32_t m = acc & 0x8000u;
        acc ^= m ^ (m >> (ex & 31u));
        // a lane past the end reads only zero bits: its plane word is zero
        // and its state stays put; keep its position inside the padding
        at = __builtin_elementwise_min(at, kMaxBits + 32u);
    }
    pos = at;
    store_plane<P>(A, acc, xv);
    return past;
}

// Planes below this one may be cut by the bit budget without the exact
// inverse lift leaving the int32 range: a cut at plane lo moves a
// coefficient by less than 2^(lo+1), the 2-D inverse lift multiplies that by
// at most 3.75^2, and the block's integers stay below 2^30 + 2^29.3 < 2^31.
constexpr int kSafeCutPlane = 26;

// `cut` ends true when the budget ended before plane kSafeCutPlane was read
// in full (the block's top planes only), else false.  `past`: the wave's
// lanes already past their budget.
template <int NW, int STRIDE, int P>
__device__ __forceinline__ void decode_planes_from(const uint32_t* lw, const uint32_t* tab, uint32_t& pos,
                                                   uint32_t& ns, uint32_t (&A)[16], bool& cut, uint64_t past)
{
    if constexpr (P >= 0) {
        if (past == __builtin_amdgcn_read_exec()) {
            // planes P..0 stay zero: words 0..P-16 were never written
            if constexpr (P >= 16) {
#pragma unroll
                for (int q = 0; q <= P - 16; ++q)
                    A[q] = 0u;
            }
            return;
        }
        past = decode_plane<NW, STRIDE, P>(lw, tab, pos, ns, A);
        if constexpr (P == kSafeCutPlane)
            cut = pos > 32u * NW;
        decode_planes_from<NW, STRIDE, P - 1>(lw, tab, pos, ns, A, cut, past);
    }
}

// Words a lane's staged block occupies in LDS: NW words of the block, then
// zeros, which the decoder reads past the end of the bit budget.  Each read
// takes words q and q + 1 of a position; a position stays below 32 bits past
// the end plus one plane (a plane never spans more than 31 bits: nsig
// verbatim bits and at most 1 + 2 (15 - nsig) section bits, or 16 verbatim
// bits), so word NW + 2 is the last one read.
template <int NW>
constexpr int kStagedWords = NW + 3;

// Decode the coefficients of the block staged at lw[q * STRIDE], q =
// 0..NW-1 (lw[q * STRIDE] == 0 for q = NW..NW+2); w0 == lw[0]; tab = the
// section table (in LDS).  Outputs the 16 transform coefficients (two's
// complement, at their block positions 4r + c, before the inverse
// transform) and emax.  Returns false for an all-zero block (then cf[] is
// all 0).  Every bit pattern decodes (the function is total).
// `cut`: the budget ended above plane kSafeCutPlane (then only the exact
// integer lift reproduces the decoded block; see lin_inv_lift).
template <int NW, int STRIDE>
__device__ __forceinline__ bool decode_block_coeffs(const uint32_t* lw, const uint32_t* tab, uint32_t w0, int& emax,
                                                    uint32_t (&cf)[16], bool& cut)
{
    const bool nz = (w0 & 1u) != 0;
    emax = (int)((w0 >> 1) & 0xFFu) - 127;
    uint32_t pos = nz ? 9u : 32u * NW; // next bit to read; decoding stops at 32*NW
    uint32_t ns = 0u;                   // nsig * kSecRow: coefficients 0..nsig-1 significant
    uint32_t A[16]; // every word is written by a plane or by the early exit
    cut = nz;       // a zero block is exact; others until plane kSafeCutPlane is read
    decode_planes_from<NW, STRIDE, 31>(lw, tab, pos, ns, A, cut, __ballot(!nz));
    transpose_planes(A);
    // negabinary -> two's complement (one v_xad each), undo the sequency
    // order
#pragma unroll
    for (int s = 0; s < 16; ++s)
        cf[order_of(s)] = nega_to_int(A[s]);
    return nz;
}

// The decoded block: its coefficients through the inverse transform, as
// integers (value = iv * 2^(emax - 30)).
template <int NW, int STRIDE>
__device__ __forceinline__ bool decode_block_coeffs(const uint32_t* lw, const uint32_t* tab, uint32_t w0, int& emax,
                                                    uint32_t (&cf)[16])
{
    bool cut;
    return decode_block_coeffs<NW, STRIDE>(lw, tab, w0, emax, cf, cut);
}

template <int NW, int STRIDE>
__device__ __forceinline__ bool decode_block_ints(const uint32_t* lw, const uint32_t* tab, uint32_t w0, int& emax,
                                                  uint32_t (&iv)[16])
{
    const bool nz = decode_block_coeffs<NW, STRIDE>(lw, tab, w0, emax, iv);
    inv_xform(iv);
    return nz;
}

// The inverse lift without its two floor halvings is a linear map B (the
// inverse of the forward lift's matrix (1/16) [[4,4,4,4],[5,1,-1,-5],
// [-4,4,4,-4],[-2,6,-6,2]]):
//   B = [[1, 3/2, -1, -1/4], [1, 1/2, 1, 5/4], [1, -1/2, 1, -5/4], [1, -3/2, -1, 1/4]]
// and the 2-D inverse transform of a coefficient block C is B C B^T up to
// those halvings (at most a few units of the block's last integer bit).
// Hence a block's row sums against u are B (C (B^T u)): B^T u is a per-
// column-block quantity, and B, being the same for every block, can be
// applied once to a row group's accumulated sums.  This holds while the
// integer lift stays inside int32; a block cut by the bit budget above plane
// kSafeCutPlane can leave it (the exact lift wraps modulo 2^32), so such
// blocks take the exact path: their decoded integers' row sums z, carried
// back to coefficient space as L z (L = B^-1, the forward lift's linear part).
template <typename T>
__device__ __forceinline__ void lin_inv_lift(T& x, T& y, T& z, T& w)
{
    y += w * T(0.5);
    w -= y * T(0.5);
    T t = y;
    y += w;
    w -= t;
    t = z;
    z += x;
    x -= t;
    t = y;
    y += z;
    z -= t;
    t = w;
    w += x;
    x -= t;
}

// B^T u for one block column (u0..u3 its four u values).
template <typename T>
__device__ __forceinline__ void lin_bt_u(T u0, T u1, T u2, T u3, T (&ut)[4])
{
    const T s03 = u0 + u3, d03 = u0 - u3, s12 = u1 + u2, d12 = u1 - u2;
    ut[0] = s03 + s12;
    ut[1] = T(1.5) * d03 + T(0.5) * d12;
    ut[2] = s12 - s03;
    ut[3] = T(1.25) * d12 - T(0.25) * d03;
}

// --------------------------------------------------------------- encoding
// Bit writer over a lane-private word array of NW words (zeroed first).
template <int NW>
struct BitSink {
    uint32_t w[NW];
    uint32_t pos;

    __device__ __forceinline__ void put(uint32_t bits, uint32_t k) // k <= 16
    {
        if (k == 0u)
            return;
        const uint32_t q = pos >> 5, o = pos & 31u;
        w[q] |= bits << o;
        if (o + k > 32u)
            w[q + 1] |= bits >> (32u - o);
        pos += k;
    }
};

// Biased exponent field F of a value.  For a normal value the binade
// exponent is e = F - 126 (|f| in [2^(e-1), 2^e)); a subnormal has F = 0 and
// e <= -126, which the clamp at -126 turns into F - 126 as well.  So
// emax = max over nonzero values of F, minus 126.
__device__ __forceinline__ uint32_t exp_field(float f) { return (__float_as_uint(f) >> 23) & 0xFFu; }

// Encode 16 values (local index 4r + c) into out (NW words).  Returns false
// if a value is NaN or Inf (the block is then written as a zero block).
template <int NW>
__device__ __forceinline__ bool encode_block(const float (&f)[16], uint32_t (&out)[NW])
{
    constexpr uint32_t kMaxBits = 32u * NW;
    BitSink<NW> sink;
#pragma unroll
    for (int k = 0; k < NW; ++k)
        sink.w[k] = 0u;
    sink.pos = 0u;
    bool finite = true, nonzero = false;
    uint32_t emax_field = 0u;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const uint32_t e = exp_field(f[v]);
        finite = finite && e != 0xFFu;
        if (f[v] != 0.0f) {
            nonzero = true;
            emax_field = e > emax_field ? e : emax_field;
        }
    }
    if (finite && nonzero) {
        const int emax = (int)emax_field - 126;
        sink.put(1u, 1u);
        sink.put((uint32_t)(emax + 127), 8u);
        uint32_t iv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v)
            iv[v] = (uint32_t)(int32_t)__builtin_truncf(__builtin_ldexpf(f[v], 30 - emax));
        fwd_xform(iv);
        uint32_t nb[16];
#pragma unroll
        for (int s = 0; s < 16; ++s)
            nb[s] = (iv[order_of(s)] + kNega) ^ kNega;
        uint32_t left = kMaxBits - 9u, nsig = 0u;
        for (int p = 31; p >= 0 && left != 0u; --p) {
            uint32_t x = 0u;
#pragma unroll
            for (int s = 0; s < 16; ++s)
                x |= ((nb[s] >> p) & 1u) << s;
            const uint32_t m = nsig < left ? nsig : left;
            sink.put(x & ((1u << m) - 1u), m);
            x >>= m;
            left -= m;
            while (nsig < 16u && left != 0u) {
                const uint32_t g = x != 0u;
                sink.put(g, 1u);
                left -= 1u;
                if (!g)
                    break;
                while (nsig < 15u && left != 0u) {
                    const uint32_t bit = x & 1u;
                    sink.put(bit, 1u);
                    left -= 1u;
                    if (bit)
                        break;
                    x >>= 1;
                    nsig += 1u;
                }
                x >>= 1;
                nsig += 1u;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NW; ++k)
        out[k] = sink.w[k];
    return finite;
}

} // namespace wh
