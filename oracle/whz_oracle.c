/*
 * whz_oracle.c -- CPU ORACLE (test infrastructure only).
 *
 * Plain, slow, obviously-correct reference for the compressed-matrix GEMV
 * y = M.u of the wafer-heat feed-forward deformation model (paper: GPU
 * Acceleration of Real-Time Control Loops, Sec. 2.1, Eq. 2).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * this library.  It shares no code, header or table with the GPU library.
 *
 * What it computes:
 *   - WHZ1: a zfp-style fixed-rate code for FP32 matrices in 4x4 blocks (the
 *     paper picks zfp in its fixed-rate mode, Sec. 4.3 "Data Compression",
 *     Table 2: exactly BPV bits per value).  The paper gives no codec
 *     internals; WHZ1 restates the published zfp method (block floating
 *     point, decorrelating lift, sequency order, negabinary, embedded
 *     bit-plane group testing) and fixes every choice.  Steps below are
 *     written bit by bit from that definition, with no blocking or fusion.
 *   - GEMV in FP64: y[i] = sum_j (double)Mhat[i,j] * (double)u[j], summed in
 *     ascending j (the plain definition of Eq. 5 in double precision).
 *   - "paper-MP" GEMV: FP32 product, FP64 running sum, FP32 result, exactly
 *     the sequential mixed-precision GEMV of Fig. 7 (Sec. 4.4).
 *
 * Integer conventions: the lifting arithmetic is two's complement modulo
 * 2^32 and ">> 1" is a floor (arithmetic) shift.  This file relies on GCC's
 * documented behaviour: signed right shift is arithmetic and conversion of
 * an out-of-range unsigned value to int32_t wraps modulo 2^32.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_SHAPE (-2)

/* ------------------------------------------------------------------ */
/* bit I/O: stream bit s is bit (s mod 8) of byte floor(s/8)          */
/* ------------------------------------------------------------------ */
typedef struct {
    uint8_t *buf;
    uint64_t pos;
} bitw;

typedef struct {
    const uint8_t *buf;
    uint64_t pos;
} bitr;

static void put_bit(bitw *w, unsigned bit)
{
    if (bit & 1u)
        w->buf[w->pos >> 3] |= (uint8_t)(1u << (w->pos & 7u));
    w->pos++;
}

static unsigned get_bit(bitr *r)
{
    unsigned bit = (r->buf[r->pos >> 3] >> (r->pos & 7u)) & 1u;
    r->pos++;
    return bit;
}

/* ------------------------------------------------------------------ */
/* the sequency order of the 16 transform coefficients                 */
/* ------------------------------------------------------------------ */
/* Coefficient at local index v = 4r + c has horizontal frequency c and
 * vertical frequency r.  Order: by c + r, then by c^2 + r^2, then larger c
 * first.  Built by a plain selection sort from that rule. */
static int order_key_less(int va, int vb)
{
    int ca = va & 3, ra = va >> 2, cb = vb & 3, rb = vb >> 2;
    if (ca + ra != cb + rb)
        return ca + ra < cb + rb;
    if (ca * ca + ra * ra != cb * cb + rb * rb)
        return ca * ca + ra * ra < cb * cb + rb * rb;
    return ca > cb;
}

static void sequency_order(int order[16])
{
    int used[16] = {0};
    for (int s = 0; s < 16; s++) {
        int best = -1;
        for (int v = 0; v < 16; v++) {
            if (used[v])
                continue;
            if (best < 0 || order_key_less(v, best))
                best = v;
        }
        used[best] = 1;
        order[s] = best;
    }
}

void orc_sequency_order(int32_t *out16)
{
    int order[16];
    sequency_order(order);
    for (int s = 0; s < 16; s++)
        out16[s] = order[s];
}

/* ------------------------------------------------------------------ */
/* decorrelating lift (modulo 2^32, floor shifts)                     */
/* ------------------------------------------------------------------ */
static int32_t add32(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
static int32_t sub32(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }
static int32_t half_floor(int32_t a) { return a >> 1; }
static int32_t twice(int32_t a) { return (int32_t)((uint32_t)a << 1); }

/* forward lift L on (x, y, z, w) = p[0], p[s], p[2s], p[3s] */
static void fwd_lift(int32_t *p, int s)
{
    int32_t x = p[0], y = p[s], z = p[2 * s], w = p[3 * s];
    x = half_floor(add32(x, w));
    w = sub32(w, x);
    z = half_floor(add32(z, y));
    y = sub32(y, z);
    x = half_floor(add32(x, z));
    z = sub32(z, x);
    w = half_floor(add32(w, y));
    y = sub32(y, w);
    w = add32(w, half_floor(y));
    y = sub32(y, half_floor(w));
    p[0] = x;
    p[s] = y;
    p[2 * s] = z;
    p[3 * s] = w;
}

/* inverse lift L^-1, the steps of L undone in reverse order */
static void inv_lift(int32_t *p, int s)
{
    int32_t x = p[0], y = p[s], z = p[2 * s], w = p[3 * s];
    y = add32(y, half_floor(w));
    w = sub32(w, half_floor(y));
    y = add32(y, w);
    w = sub32(twice(w), y);
    z = add32(z, x);
    x = sub32(twice(x), z);
    y = add32(y, z);
    z = sub32(twice(z), y);
    w = add32(w, x);
    x = sub32(twice(x), w);
    p[0] = x;
    p[s] = y;
    p[2 * s] = z;
    p[3 * s] = w;
}

void orc_fwd_lift4(int32_t *v4) { fwd_lift(v4, 1); }
void orc_inv_lift4(int32_t *v4) { inv_lift(v4, 1); }

/* 2-D forward transform: L along each block row (over c), then along each
 * block column (over r).  Local index v = 4r + c. */
static void fwd_xform(int32_t b[16])
{
    for (int r = 0; r < 4; r++)
        fwd_lift(b + 4 * r, 1);
    for (int c = 0; c < 4; c++)
        fwd_lift(b + c, 4);
}

/* 2-D inverse transform: exact reverse order (columns first, then rows). */
static void inv_xform(int32_t b[16])
{
    for (int c = 0; c < 4; c++)
        inv_lift(b + c, 4);
    for (int r = 0; r < 4; r++)
        inv_lift(b + 4 * r, 1);
}

void orc_fwd_xform(int32_t *b16) { fwd_xform(b16); }
void orc_inv_xform(int32_t *b16) { inv_xform(b16); }

/* ------------------------------------------------------------------ */
/* negabinary                                                          */
/* ------------------------------------------------------------------ */
static uint32_t to_negabinary(int32_t i) { return ((uint32_t)i + 0xAAAAAAAAu) ^ 0xAAAAAAAAu; }
static int32_t from_negabinary(uint32_t n) { return (int32_t)((n ^ 0xAAAAAAAAu) - 0xAAAAAAAAu); }

/* ------------------------------------------------------------------ */
/* embedded bit-plane coder on 16 unsigned coefficients                */
/* ------------------------------------------------------------------ */
/* Writes planes 31 down to `lo`, at most `budget` bits; returns the number
 * written. */
static unsigned encode_planes(bitw *w, const uint32_t n16[16], unsigned budget, int lo)
{
    unsigned left = budget;
    unsigned nsig = 0; /* coefficients 0..nsig-1 are significant */
    for (int p = 31; p >= lo && left > 0; p--) {
        uint32_t x = 0;
        for (int s = 0; s < 16; s++)
            x |= ((n16[s] >> p) & 1u) << s;
        /* (i) the bits of the already-significant coefficients, verbatim */
        unsigned m = nsig < left ? nsig : left;
        for (unsigned k = 0; k < m; k++)
            put_bit(w, (x >> k) & 1u);
        left -= m;
        x >>= m;
        /* (ii) group tests locating the newly significant coefficients */
        while (nsig < 16 && left > 0) {
            unsigned g = x != 0;
            put_bit(w, g);
            left--;
            if (!g)
                break;
            while (nsig < 15 && left > 0) {
                unsigned bit = x & 1u;
                put_bit(w, bit);
                left--;
                if (bit)
                    break;
                x >>= 1;
                nsig++;
            }
            x >>= 1;
            nsig++;
        }
    }
    return budget - left;
}

/* Reads planes 31 down to `lo`, at most `budget` bits, into n16 (zeroed
 * first; planes below lo stay zero); returns bits read. */
static unsigned decode_planes(bitr *r, uint32_t n16[16], unsigned budget, int lo)
{
    unsigned left = budget;
    unsigned nsig = 0;
    for (int s = 0; s < 16; s++)
        n16[s] = 0;
    for (int p = 31; p >= lo && left > 0; p--) {
        uint32_t x = 0;
        unsigned m = nsig < left ? nsig : left;
        for (unsigned k = 0; k < m; k++)
            x |= (uint32_t)get_bit(r) << k;
        left -= m;
        while (nsig < 16 && left > 0) {
            unsigned g = get_bit(r);
            left--;
            if (!g)
                break;
            while (nsig < 15 && left > 0) {
                unsigned bit = get_bit(r);
                left--;
                if (bit)
                    break;
                nsig++;
            }
            /* the run ended: on a read 1, at position 15, or with the
             * budget spent -- in every case coefficient nsig gets bit p */
            x |= 1u << nsig;
            nsig++;
        }
        for (int s = 0; s < 16; s++)
            n16[s] |= ((x >> s) & 1u) << p;
    }
    return budget - left;
}

/* Coder-level entry points (for tests of the coder alone). */
unsigned orc_encode_planes(const uint32_t *n16, unsigned budget, uint8_t *out)
{
    bitw w = {out, 0};
    return encode_planes(&w, n16, budget, 0);
}

unsigned orc_decode_planes(const uint8_t *in, unsigned budget, uint32_t *n16)
{
    bitr r = {in, 0};
    return decode_planes(&r, n16, budget, 0);
}

/* ------------------------------------------------------------------ */
/* one 4x4 block                                                       */
/* ------------------------------------------------------------------ */
/* exponent e with |f| in [2^(e-1), 2^e) */
static int binade(float f)
{
    int e;
    frexp((double)f, &e);
    return e;
}

/* The block-floating-point step, the forward transform, the sequency
 * order and negabinary: f[16] (local index 4r + c) -> n16[16] and emax.
 * Returns 0 for an all-zero block, 1 otherwise, ORC_ERR_INVALID on NaN/Inf. */
static int block_to_negabinary(const float f[16], int *emax_out, uint32_t n16[16])
{
    int nonzero = 0, emax = -126;
    for (int v = 0; v < 16; v++) {
        if (isnan(f[v]) || isinf(f[v]))
            return ORC_ERR_INVALID;
        if (f[v] != 0.0f) {
            int e = binade(f[v]);
            if (!nonzero || e > emax)
                emax = e;
            nonzero = 1;
        }
    }
    if (!nonzero)
        return 0;
    if (emax < -126)
        emax = -126;
    /* block floating point: exact scaling, truncation toward zero */
    int32_t iblk[16];
    double scale = ldexp(1.0, 30 - emax);
    for (int v = 0; v < 16; v++)
        iblk[v] = (int32_t)trunc((double)f[v] * scale);
    fwd_xform(iblk);
    int order[16];
    sequency_order(order);
    for (int s = 0; s < 16; s++)
        n16[s] = to_negabinary(iblk[order[s]]);
    *emax_out = emax;
    return 1;
}

/* n16[16] and emax -> f[16]: negabinary, sequency order and transform
 * undone, f = ldexp(RNE_f32(i), emax - 30) (the double product is exact,
 * the final conversion is the one IEEE rounding). */
static void negabinary_to_block(const uint32_t n16[16], int emax, float f[16])
{
    int order[16];
    sequency_order(order);
    int32_t iblk[16];
    for (int s = 0; s < 16; s++)
        iblk[order[s]] = from_negabinary(n16[s]);
    inv_xform(iblk);
    for (int v = 0; v < 16; v++) {
        float fi = (float)iblk[v];
        f[v] = (float)((double)fi * ldexp(1.0, emax - 30));
    }
}

static void put_header(bitw *w, int emax)
{
    unsigned E = (unsigned)(emax + 127);
    put_bit(w, 1);
    for (int k = 0; k < 8; k++)
        put_bit(w, (E >> k) & 1u);
}

static int get_exponent(bitr *r)
{
    unsigned E = 0;
    for (int k = 0; k < 8; k++)
        E |= get_bit(r) << k;
    return (int)E - 127;
}

/* Encode f[16] (local index 4r + c) into exactly maxbits bits at w->pos.
 * Returns ORC_ERR_INVALID on NaN/Inf. */
static int encode_block(bitw *w, const float f[16], unsigned maxbits)
{
    uint64_t start = w->pos;
    int emax = 0;
    uint32_t n16[16];
    int st = block_to_negabinary(f, &emax, n16);
    if (st < 0)
        return st;
    if (st == 0) {
        put_bit(w, 0);
    } else {
        put_header(w, emax);
        encode_planes(w, n16, maxbits - 9, 0);
    }
    w->pos = start + maxbits; /* pad: unused bits stay zero */
    return ORC_OK;
}

/* Decode exactly maxbits bits at r->pos into f[16] (local index 4r + c).
 * Total: any bit pattern decodes. */
static void decode_block(bitr *r, float f[16], unsigned maxbits)
{
    uint64_t start = r->pos;
    if (!get_bit(r)) {
        for (int v = 0; v < 16; v++)
            f[v] = 0.0f;
    } else {
        int emax = get_exponent(r);
        uint32_t n16[16];
        decode_planes(r, n16, maxbits - 9, 0);
        negabinary_to_block(n16, emax, f);
    }
    r->pos = start + maxbits;
}

/* ------------------------------------------------------------------ */
/* matrix-level codec                                                  */
/* ------------------------------------------------------------------ */
static int check_shape(uint32_t rows, uint32_t cols, uint32_t rate)
{
    if (rate < 1 || rate > 64)
        return ORC_ERR_INVALID;
    if (rows == 0 || cols == 0)
        return ORC_ERR_SHAPE;
    return ORC_OK;
}

/* Blocks along a dimension of n values: the last one may be partial. */
static uint32_t nblk(uint32_t n) { return (n + 3) / 4; }

/* Index n-1 for positions past the end: a partial block is completed by
 * repeating the matrix's last row / column (edge padding). */
static uint32_t clamp_index(uint32_t i, uint32_t n) { return i < n ? i : n - 1; }

/* M: rows x cols FP32 row-major.  stream: nblk(rows)*nblk(cols)*2*rate
 * bytes, zeroed by this call.  Block (bi, bj) is block number
 * bi*nblk(cols) + bj; a partial block holds the edge-padded values. */
int orc_encode(const float *M, uint32_t rows, uint32_t cols, uint32_t rate, uint8_t *stream)
{
    int st = check_shape(rows, cols, rate);
    if (st)
        return st;
    unsigned maxbits = 16u * rate;
    uint64_t nbytes = (uint64_t)nblk(rows) * nblk(cols) * (maxbits / 8);
    memset(stream, 0, nbytes);
    bitw w = {stream, 0};
    for (uint32_t bi = 0; bi < nblk(rows); bi++) {
        for (uint32_t bj = 0; bj < nblk(cols); bj++) {
            float f[16];
            for (int r = 0; r < 4; r++)
                for (int c = 0; c < 4; c++)
                    f[4 * r + c] = M[(uint64_t)clamp_index(4 * bi + r, rows) * cols + clamp_index(4 * bj + c, cols)];
            st = encode_block(&w, f, maxbits);
            if (st)
                return st;
        }
    }
    return ORC_OK;
}

/* Decode blocks [b0, b0 + nblocks) of a stream of the given rate into
 * out[nblocks][16] (local index 4r + c).  maxbits = 16 * rate. */
int orc_decode_blocks(const uint8_t *stream, uint32_t rate, uint64_t b0, uint64_t nblocks, float *out)
{
    if (rate < 1 || rate > 64)
        return ORC_ERR_INVALID;
    unsigned maxbits = 16u * rate;
    bitr r = {stream, b0 * maxbits};
    for (uint64_t b = 0; b < nblocks; b++)
        decode_block(&r, out + 16 * b, maxbits);
    return ORC_OK;
}

/* Decode a whole matrix into Mhat (rows x cols row-major); the padding of
 * partial blocks is dropped. */
int orc_decode(const uint8_t *stream, uint32_t rows, uint32_t cols, uint32_t rate, float *Mhat)
{
    int st = check_shape(rows, cols, rate);
    if (st)
        return st;
    unsigned maxbits = 16u * rate;
    bitr r = {stream, 0};
    for (uint32_t bi = 0; bi < nblk(rows); bi++) {
        for (uint32_t bj = 0; bj < nblk(cols); bj++) {
            float f[16];
            decode_block(&r, f, maxbits);
            for (uint32_t rr = 0; rr < 4; rr++)
                for (uint32_t c = 0; c < 4; c++)
                    if (4 * bi + rr < rows && 4 * bj + c < cols)
                        Mhat[(uint64_t)(4 * bi + rr) * cols + 4 * bj + c] = f[4 * rr + c];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* variable-rate modes: fixed precision, fixed accuracy (Sec. 4.3)      */
/* ------------------------------------------------------------------ */
/* The same block code with no bit budget: a nonzero block codes bit planes
 * 31 down to 32 - P and ends there (its length follows from its bits).
 *   fixed precision (mode 0, param = P in 1..32): P planes in every block;
 *   fixed accuracy (mode 1, param = minexp, tolerance 2^minexp):
 *     P = clamp(emax - minexp + 7, 0, 32).  Dropping the planes below
 *     32 - P changes each coefficient by less than (2/3) 2^(32-P) units of
 *     2^(emax-30); the inverse transform's row and column gain (3.75 each)
 *     carries that to under 0.3 tol per value, and the truncation to
 *     integers and the lift's floor shifts add a few units of 2^(emax-30),
 *     so |error| <= tol whenever P < 32 is not clamped (emax - minexp <= 25).
 * Blocks follow each other with no padding, in raster order.  The index
 * holds the bit offset of every ORC_GROUP-th block of each block row:
 * index[bi * ngroups + a] = offset of block (bi, ORC_GROUP * a). */
enum { ORC_VAR_PRECISION = 0, ORC_VAR_ACCURACY = 1 };
#define ORC_GROUP 32u

static int var_planes(int mode, int param, int emax)
{
    if (mode == ORC_VAR_PRECISION)
        return param;
    int p = emax - param + 7;
    return p < 0 ? 0 : p > 32 ? 32 : p;
}

static int check_var(int mode, int param)
{
    if (mode == ORC_VAR_PRECISION)
        return param >= 1 && param <= 32 ? ORC_OK : ORC_ERR_INVALID;
    if (mode == ORC_VAR_ACCURACY)
        return param >= -160 && param <= 160 ? ORC_OK : ORC_ERR_INVALID;
    return ORC_ERR_INVALID;
}

static int encode_block_var(bitw *w, const float f[16], int mode, int param)
{
    int emax = 0;
    uint32_t n16[16];
    int st = block_to_negabinary(f, &emax, n16);
    if (st < 0)
        return st;
    if (st == 0) {
        put_bit(w, 0);
        return ORC_OK;
    }
    put_header(w, emax);
    encode_planes(w, n16, ~0u, 32 - var_planes(mode, param, emax));
    return ORC_OK;
}

static void decode_block_var(bitr *r, float f[16], int mode, int param)
{
    if (!get_bit(r)) {
        for (int v = 0; v < 16; v++)
            f[v] = 0.0f;
        return;
    }
    int emax = get_exponent(r);
    uint32_t n16[16];
    decode_planes(r, n16, ~0u, 32 - var_planes(mode, param, emax));
    negabinary_to_block(n16, emax, f);
}

uint32_t orc_var_groups(uint32_t cols) { return (nblk(cols) + ORC_GROUP - 1) / ORC_GROUP; }

/* Most bits a block can take: header, then per plane the verbatim bits of
 * the significant coefficients, one group test and the run bits. */
uint64_t orc_var_capacity_bytes(uint32_t rows, uint32_t cols)
{
    return (uint64_t)nblk(rows) * nblk(cols) * ((9 + 32 * 33 + 7) / 8) + 16;
}

/* M: rows x cols FP32 -> stream (cap bytes, zeroed here) and index
 * (nblk(rows) * orc_var_groups(cols) entries); *nbits = bits written. */
int orc_encode_var(const float *M, uint32_t rows, uint32_t cols, int mode, int param, uint8_t *stream, uint64_t cap,
                   uint64_t *index, uint64_t *nbits)
{
    if (rows == 0 || cols == 0)
        return ORC_ERR_SHAPE;
    if (check_var(mode, param) || cap < orc_var_capacity_bytes(rows, cols))
        return ORC_ERR_INVALID;
    memset(stream, 0, cap);
    bitw w = {stream, 0};
    uint32_t ng = orc_var_groups(cols);
    for (uint32_t bi = 0; bi < nblk(rows); bi++) {
        for (uint32_t bj = 0; bj < nblk(cols); bj++) {
            if (bj % ORC_GROUP == 0)
                index[(uint64_t)bi * ng + bj / ORC_GROUP] = w.pos;
            float f[16];
            for (int r = 0; r < 4; r++)
                for (int c = 0; c < 4; c++)
                    f[4 * r + c] = M[(uint64_t)clamp_index(4 * bi + r, rows) * cols + clamp_index(4 * bj + c, cols)];
            int st = encode_block_var(&w, f, mode, param);
            if (st)
                return st;
        }
    }
    *nbits = w.pos;
    return ORC_OK;
}

/* Decode into Mhat (rows x cols).  With an index each group of blocks
 * starts at its recorded offset; with index == NULL the blocks are read one
 * after another from bit 0. */
int orc_decode_var(const uint8_t *stream, const uint64_t *index, uint32_t rows, uint32_t cols, int mode, int param,
                   float *Mhat)
{
    if (rows == 0 || cols == 0)
        return ORC_ERR_SHAPE;
    if (check_var(mode, param))
        return ORC_ERR_INVALID;
    bitr r = {stream, 0};
    uint32_t ng = orc_var_groups(cols);
    for (uint32_t bi = 0; bi < nblk(rows); bi++) {
        for (uint32_t bj = 0; bj < nblk(cols); bj++) {
            if (index && bj % ORC_GROUP == 0)
                r.pos = index[(uint64_t)bi * ng + bj / ORC_GROUP];
            float f[16];
            decode_block_var(&r, f, mode, param);
            for (uint32_t rr = 0; rr < 4; rr++)
                for (uint32_t c = 0; c < 4; c++)
                    if (4 * bi + rr < rows && 4 * bj + c < cols)
                        Mhat[(uint64_t)(4 * bi + rr) * cols + 4 * bj + c] = f[4 * rr + c];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* GEMV over the decoded matrix, one block-row at a time                */
/* ------------------------------------------------------------------ */
enum { ORC_MODE_FP64 = 0, ORC_MODE_PAPER_MP = 1 };

typedef struct {
    const uint8_t *stream;
    uint32_t rows, cols, rate;
    const float *u;
    uint32_t bi_begin, bi_end; /* block-rows handled by this worker */
    uint32_t row0;             /* first output row of the call */
    int mode;
    double *y64;  /* FP64 mode output, indexed by row - row0 */
    float *y32;   /* paper-MP output */
} gemv_job;

static void *gemv_worker(void *arg)
{
    gemv_job *job = (gemv_job *)arg;
    uint32_t cols = job->cols, padded = 4 * nblk(cols);
    unsigned maxbits = 16u * job->rate;
    float *rowbuf = (float *)malloc(sizeof(float) * 4 * (size_t)padded);
    if (!rowbuf)
        return (void *)1;
    for (uint32_t bi = job->bi_begin; bi < job->bi_end; bi++) {
        bitr r = {job->stream, (uint64_t)bi * nblk(cols) * maxbits};
        for (uint32_t bj = 0; bj < nblk(cols); bj++) {
            float f[16];
            decode_block(&r, f, maxbits);
            for (int rr = 0; rr < 4; rr++)
                for (int c = 0; c < 4; c++)
                    rowbuf[(size_t)rr * padded + 4 * bj + c] = f[4 * rr + c];
        }
        for (uint32_t rr = 0; rr < 4 && 4 * bi + rr < job->rows; rr++) {
            if (4 * bi + rr < job->row0) /* before the range, in its first block row */
                continue;
            /* the sum runs over the matrix's own columns only */
            const float *m = rowbuf + (size_t)rr * padded;
            uint32_t row = 4 * bi + rr - job->row0;
            if (job->mode == ORC_MODE_FP64) {
                double sum = 0.0;
                for (uint32_t j = 0; j < cols; j++)
                    sum += (double)m[j] * (double)job->u[j];
                job->y64[row] = sum;
            } else {
                double sum = 0.0;
                for (uint32_t j = 0; j < cols; j++) {
                    float product = m[j] * job->u[j];
                    sum += (double)product;
                }
                job->y32[row] = (float)sum;
            }
        }
    }
    free(rowbuf);
    return NULL;
}

static int run_gemv(const uint8_t *stream, uint32_t rows, uint32_t cols, uint32_t rate, const float *u,
                    uint32_t row_begin, uint32_t row_end, int mode, double *y64, float *y32, int nthreads)
{
    int st = check_shape(rows, cols, rate);
    if (st)
        return st;
    /* any range of rows: its first and last block rows are decoded whole */
    if (row_begin > row_end || row_end > rows)
        return ORC_ERR_SHAPE;
    uint32_t nbr = row_begin < row_end ? nblk(row_end) - row_begin / 4 : 0;
    if (nthreads < 1)
        nthreads = 1;
    if ((uint32_t)nthreads > nbr)
        nthreads = nbr ? (int)nbr : 1;
    gemv_job *jobs = (gemv_job *)calloc((size_t)nthreads, sizeof(gemv_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return ORC_ERR_INVALID;
    }
    int failed = 0;
    for (int t = 0; t < nthreads; t++) {
        gemv_job *j = &jobs[t];
        j->stream = stream;
        j->rows = row_end;
        j->cols = cols;
        j->rate = rate;
        j->u = u;
        j->bi_begin = row_begin / 4 + (uint32_t)((uint64_t)nbr * t / nthreads);
        j->bi_end = row_begin / 4 + (uint32_t)((uint64_t)nbr * (t + 1) / nthreads);
        j->row0 = row_begin;
        j->mode = mode;
        j->y64 = y64;
        j->y32 = y32;
        if (nthreads == 1) {
            failed |= gemv_worker(j) != NULL;
        } else if (pthread_create(&tids[t], NULL, gemv_worker, j) != 0) {
            failed = 1;
            tids[t] = 0;
        }
    }
    if (nthreads > 1) {
        for (int t = 0; t < nthreads; t++) {
            void *ret = NULL;
            if (tids[t]) {
                pthread_join(tids[t], &ret);
                failed |= ret != NULL;
            }
        }
    }
    free(jobs);
    free(tids);
    return failed ? ORC_ERR_INVALID : ORC_OK;
}

/* y[i - row_begin] = sum_j (double)Mhat[i,j] * (double)u[j], ascending j. */
int orc_gemv_fp64(const uint8_t *stream, uint32_t rows, uint32_t cols, uint32_t rate, const float *u,
                  uint32_t row_begin, uint32_t row_end, double *y, int nthreads)
{
    return run_gemv(stream, rows, cols, rate, u, row_begin, row_end, ORC_MODE_FP64, y, NULL, nthreads);
}

/* Fig. 7 semantics: product = (float)Mhat*u, sum += (double)product,
 * y = (float)sum. */
int orc_gemv_paper_mp(const uint8_t *stream, uint32_t rows, uint32_t cols, uint32_t rate, const float *u,
                      uint32_t row_begin, uint32_t row_end, float *y, int nthreads)
{
    return run_gemv(stream, rows, cols, rate, u, row_begin, row_end, ORC_MODE_PAPER_MP, NULL, y, nthreads);
}

/* Dense FP64 GEMV over an uncompressed FP32 matrix (rows x cols). */
void orc_dense_gemv_fp64(const float *M, uint32_t rows, uint32_t cols, const float *u, double *y)
{
    for (uint32_t i = 0; i < rows; i++) {
        double sum = 0.0;
        for (uint32_t j = 0; j < cols; j++)
            sum += (double)M[(uint64_t)i * cols + j] * (double)u[j];
        y[i] = sum;
    }
}

/* Dense paper-MP GEMV (Fig. 7) over an uncompressed FP32 matrix. */
void orc_dense_gemv_paper_mp(const float *M, uint32_t rows, uint32_t cols, const float *u, float *y)
{
    for (uint32_t i = 0; i < rows; i++) {
        double sum = 0.0;
        for (uint32_t j = 0; j < cols; j++) {
            float product = M[(uint64_t)i * cols + j] * u[j];
            sum += (double)product;
        }
        y[i] = (float)sum;
    }
}

/* Naive sequential FP32 accumulation (the precision loss the paper warns
 * about for a 256000-term row, Sec. 4.4): product and sum both in FP32. */
void orc_dense_gemv_fp32_naive(const float *M, uint32_t rows, uint32_t cols, const float *u, float *y)
{
    for (uint32_t i = 0; i < rows; i++) {
        float sum = 0.0f;
        for (uint32_t j = 0; j < cols; j++) {
            float product = M[(uint64_t)i * cols + j] * u[j];
            sum = sum + product;
        }
        y[i] = sum;
    }
}
