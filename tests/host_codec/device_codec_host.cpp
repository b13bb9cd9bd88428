// Host build of the GPU codec (whz_device.hpp) for CPU tests: the same
// decoder and encoder source, with the few AMDGPU builtins it uses written
// out from their ISA definitions, one block per "lane".
//
//   device_codec_host decode <nw> <nblocks> <in> <out> [idle]
//       in: nblocks * nw uint32 words; out: nblocks * 16 float32
//       idle = 1: wave votes report other lanes still busy at random, so the
//       decoder's loops take extra trips with this lane finished (as lanes
//       of a wave do on the GPU)
//   device_codec_host linear 0 <nblocks> <in> <out>
//       in: nblocks * (16 int32 coefficients at positions 4r + c, then 4
//       float32 u); out: nblocks * 8 float64: the block's four row sums
//       against u through the exact integer inverse transform, then through
//       the linear form B (C (B^T u)) that the fused kernels use
//   device_codec_host encode <nw> <nblocks> <in> <out>
//       in: nblocks * 16 float32 (v = 4r + c); out: nblocks * nw words;
//       exit status = number of blocks with NaN/Inf (encoded as zero)
//
// Each staged block gets exactly the LDS words the GPU kernels give it (nw
// words then the zero padding, kStagedWords), in its own heap allocation, so
// an AddressSanitizer build reports any read past that padding.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#define __device__
#define __host__
#define __forceinline__ inline
#define __builtin_elementwise_min(a, b) ((a) < (b) ? (a) : (b))

static bool g_idle_lanes = false;
static uint64_t g_lcg = 1;

// v_alignbit_b32: ({hi, lo} >> (sh & 31)) low 32 bits
static inline uint32_t __builtin_amdgcn_alignbit(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (sh & 31u));
}
// v_bfe_u32: w bits of v from bit off (offset and width taken mod 32, as the ISA does)
static inline uint32_t __builtin_amdgcn_ubfe(uint32_t v, uint32_t off, uint32_t w)
{
    off &= 31u;
    w &= 31u;
    return w == 0 ? 0u : (v >> off) & ((1u << w) - 1u);
}
// v_perm_b32: byte i of the result = byte sel_i of {s0, s1} (s1 = bytes 0..3);
// selectors 12 and 13+ give 0x00 and 0xFF (8..11 are sign replications, unused)
static inline uint32_t __builtin_amdgcn_perm(uint32_t s0, uint32_t s1, uint32_t sel)
{
    const uint64_t d = ((uint64_t)s0 << 32) | s1;
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t b = (sel >> (8 * i)) & 0xFFu;
        const uint32_t v = b < 8 ? (uint32_t)((d >> (8 * b)) & 0xFFu) : (b == 12 ? 0u : 0xFFu);
        r |= v << (8 * i);
    }
    return r;
}
static inline uint32_t coin()
{
    g_lcg = g_lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(g_lcg >> 63);
}
// wave vote of a one-lane wave; with idle lanes, "some other lane is still
// busy" half the time when this lane's predicate is false
static inline int __any(int p)
{
    if (p || !g_idle_lanes)
        return p;
    return (int)coin();
}
// the active lanes: this lane (bit 0) and, with idle lanes, one more (bit 1)
static inline uint64_t __builtin_amdgcn_read_exec() { return g_idle_lanes ? 3u : 1u; }
// ballot over the active lanes; the other lane's predicate is a coin toss
static inline uint64_t __ballot(int p)
{
    uint64_t m = p ? 1u : 0u;
    if (g_idle_lanes)
        m |= (uint64_t)coin() << 1;
    return m;
}
// v_sub_u32 with clamp: a - b, or 0 where b > a
#define __builtin_elementwise_sub_sat(a, b) ((a) > (b) ? (a) - (b) : 0u)
static inline uint32_t __float_as_uint(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

#include "../../paper_1902_08018_amd/csrc/whz_device.hpp"

template <int NW>
static void decode(const uint32_t* words, size_t n, float* out)
{
    static const wh::SectionTable table{};
    for (size_t b = 0; b < n; ++b) {
        std::vector<uint32_t> lw(wh::kStagedWords<NW>, 0u);
        std::memcpy(lw.data(), words + b * NW, 4 * NW);
        int emax;
        uint32_t iv[16];
        wh::decode_block_ints<NW, 1>(lw.data(), table.e, lw[0], emax, iv);
        for (int v = 0; v < 16; ++v)
            out[16 * b + v] = std::ldexp((float)(int32_t)iv[v], emax - 30);
    }
}

template <int NW>
static int encode(const float* blocks, size_t n, uint32_t* out)
{
    int bad = 0;
    for (size_t b = 0; b < n; ++b) {
        float f[16];
        std::memcpy(f, blocks + 16 * b, sizeof f);
        uint32_t o[NW];
        if (!wh::encode_block<NW>(f, o))
            ++bad;
        std::memcpy(out + b * NW, o, 4 * NW);
    }
    return bad;
}

template <int NW>
static int run(bool dec, size_t n, const std::vector<char>& in, std::vector<char>& out)
{
    if (dec) {
        out.resize(n * 64);
        decode<NW>(reinterpret_cast<const uint32_t*>(in.data()), n, reinterpret_cast<float*>(out.data()));
        return 0;
    }
    out.resize(n * 4 * NW);
    return encode<NW>(reinterpret_cast<const float*>(in.data()), n, reinterpret_cast<uint32_t*>(out.data()));
}

static void linear(const char* in, size_t n, double* out)
{
    for (size_t b = 0; b < n; ++b) {
        const char* rec = in + b * 80;
        uint32_t cf[16];
        float u[4];
        std::memcpy(cf, rec, 64);
        std::memcpy(u, rec + 64, 16);
        uint32_t iv[16];
        std::memcpy(iv, cf, 64);
        wh::inv_xform(iv);
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int c = 0; c < 4; ++c)
                s += (double)(int32_t)iv[4 * r + c] * (double)u[c];
            out[8 * b + r] = s;
        }
        double ut[4]; // in FP64: the test isolates the floor halvings
        wh::lin_bt_u<double>(u[0], u[1], u[2], u[3], ut);
        double v[4];
        for (int r = 0; r < 4; ++r) {
            v[r] = 0.0;
            for (int c = 0; c < 4; ++c)
                v[r] += (double)(int32_t)cf[4 * r + c] * ut[c];
        }
        wh::lin_inv_lift<double>(v[0], v[1], v[2], v[3]);
        for (int r = 0; r < 4; ++r)
            out[8 * b + 4 + r] = v[r];
    }
}

int main(int argc, char** argv)
{
    if (argc < 6) {
        std::fprintf(stderr, "usage: %s decode|encode nw nblocks in out [idle]\n", argv[0]);
        return 255;
    }
    const bool dec = std::strcmp(argv[1], "decode") == 0;
    const bool lin = std::strcmp(argv[1], "linear") == 0;
    const int nw = std::atoi(argv[2]);
    const size_t n = std::strtoull(argv[3], nullptr, 10);
    g_idle_lanes = argc > 6 && std::atoi(argv[6]) != 0;
    FILE* f = std::fopen(argv[4], "rb");
    if (!f)
        return 254;
    std::vector<char> in(lin ? n * 80 : dec ? n * 4 * nw : n * 64);
    const size_t got = std::fread(in.data(), 1, in.size(), f);
    std::fclose(f);
    if (got != in.size())
        return 253;
    std::vector<char> out;
    int rc = 0;
    if (lin) {
        out.resize(n * 64);
        linear(in.data(), n, reinterpret_cast<double*>(out.data()));
    } else switch (nw) {
    case 1: rc = run<1>(dec, n, in, out); break;
    case 2: rc = run<2>(dec, n, in, out); break;
    case 3: rc = run<3>(dec, n, in, out); break;
    case 4: rc = run<4>(dec, n, in, out); break;
    case 5: rc = run<5>(dec, n, in, out); break;
    case 6: rc = run<6>(dec, n, in, out); break;
    case 7: rc = run<7>(dec, n, in, out); break;
    case 8: rc = run<8>(dec, n, in, out); break;
    case 10: rc = run<10>(dec, n, in, out); break;
    case 12: rc = run<12>(dec, n, in, out); break;
    case 16: rc = run<16>(dec, n, in, out); break;
    default: return 252;
    }
    f = std::fopen(argv[5], "wb");
    if (!f || std::fwrite(out.data(), 1, out.size(), f) != out.size())
        return 251;
    std::fclose(f);
    return rc;
}
