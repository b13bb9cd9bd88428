/*
 * wh.h -- C ABI of libwh: on-the-fly decompression + mixed-precision GEMV
 * for very large dense model matrices on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper: "GPU Acceleration of Real-Time Control Loops",
 * Bamakhrama et al., ECRTS 2019):
 *   - Sec. 2.1, Eq. 2: the deformation model is a dense matrix-vector
 *     product Delta_d = C_d . S_{k+1}, evaluated every light-stage
 *     millisecond; all real data are single precision.
 *   - Sec. 2.1 (field/slit divide and conquer) and Fig. 2: the product
 *     uses a resident sub-matrix and a subset of its rows each millisecond.
 *   - Sec. 4.3: the matrix is stored zfp-compressed (fixed-rate mode:
 *     exactly BPV bits per value) and encoded offline.
 *   - Sec. 4.4, Eq. 5, Fig. 7: mixed-precision GEMV -- FP32 inputs and
 *     outputs, FP32 multiplies, a wide (FP64) reduction.
 *   - Sec. 1: a firm real-time loop; Sec. 2.1, Fig. 2: one product per
 *     light-stage millisecond, so every step has a deadline.
 *
 * Conventions (every entry point):
 *   - Returns a wh_status; no C++ exception crosses the ABI.  Out-params are
 *     written only when WH_OK is returned.
 *   - Pointers named d_* are device pointers (HIP/torch allocations on the
 *     context's device); other pointers are host pointers.  `stream` is a
 *     hipStream_t (NULL = the null stream).  GEMV/decode/encode calls are
 *     asynchronous and stream-ordered: argument errors are returned at once;
 *     a failed launch puts the context into a sticky failed state in which
 *     every later call returns WH_ERR_DEVICE.
 *   - The caller owns every d_* buffer it passes; the library owns its
 *     workspaces and any matrix it copied in (WH_HOST).
 *   - Matrices are row-major, rows x cols.  The compressed format takes any
 *     rows, cols >= 1: a partial 4x4 block at the bottom or right edge is
 *     coded as if the matrix were extended by repeating its last row and
 *     column (edge padding), and every output stops at the matrix's edge.
 *     Dense formats need rows and cols to be multiples of 4
 *     (else WH_ERR_SHAPE).
 *   - A context is used from one host thread at a time, except wh_submit /
 *     wh_poll which are thread-safe.
 */
#ifndef WH_H_
#define WH_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wh_status;
#define WH_OK 0
#define WH_PENDING 1
#define WH_ERR_INVALID (-1)   /* bad argument (NULL, range, unsupported)  */
#define WH_ERR_SHAPE (-2)     /* bad dimensions / row range / mismatch     */
#define WH_ERR_FORMAT (-3)    /* unknown format / rate / byte count        */
#define WH_ERR_NOMEM (-4)     /* device allocation failed                  */
#define WH_ERR_BUDGET (-5)    /* serving admission: over the HBM budget    */
#define WH_ERR_DEVICE (-6)    /* HIP error; the context is now failed      */
#define WH_ERR_NOT_FOUND (-7) /* unknown matrix handle or ticket           */
#define WH_ERR_SCRATCH (-8)   /* wh_gemv_noalloc: the call needs more than
                                 WH_NOALLOC_SCRATCH_BYTES of workspace      */

/* Storage formats of a resident matrix. */
typedef enum {
    /* WHZ1: zfp-style fixed-rate code of FP32 values in 4x4 blocks (block
     * floating point, decorrelating lift, sequency order, negabinary,
     * embedded bit-plane group testing).  Exactly 16*rate bits per block,
     * blocks in raster order b = (i/4)*ceil(cols/4) + (j/4), partial
     * blocks edge-padded.  Sec. 4.3, Table 2 ("fixed rate"). */
    WH_FMT_ZFP_FIXED_RATE = 1,
    WH_FMT_F32 = 2,          /* dense FP32, row-major                       */
    WH_FMT_F16 = 3,          /* dense IEEE half, RNE from FP32              */
    WH_FMT_BF16 = 4,         /* dense bfloat16, RNE from FP32               */
    WH_FMT_FP8E4M3_BS4 = 5,  /* OCP FP8 e4m3 codes, 4x4-block tiled (16 B per
                              * block, raster block order, v = 4r + c inside),
                              * followed by one FP32 scale per block */
    /* Variable-rate WHZ1 (Sec. 4.3, Table 2: zfp's fixed-precision and
     * fixed-accuracy modes): the same block code with no bit budget; a
     * nonzero block codes planes 31 down to 32 - P and ends there, blocks
     * follow one another with no padding.  Storage: an index of
     * ceil(rows/4) x ceil(ceil(cols/4)/32) uint64 (the bit offset, in the
     * code, of every 32nd block of each block row), then the code bytes, then
     * at least 16 zero bytes, to a multiple of 8; wh_encode_var writes it.  Any total size >= the index +
     * 16 and a multiple of 4 is accepted by wh_load_compressed (the decoder
     * reads zeros past the end). */
    WH_FMT_ZFP_FIXED_PRECISION = 6, /* desc.rate = P, 1..32 planes per block */
    WH_FMT_ZFP_FIXED_ACCURACY = 7   /* desc.rate = minexp + 1024 (tolerance
                                     * 2^minexp, minexp in -160..160):
                                     * P = clamp(emax - minexp + 7, 0, 32),
                                     * so |error| <= tolerance wherever
                                     * emax - minexp <= 25 */
} wh_format;

typedef struct {
    uint32_t rows, cols;
    int32_t fmt;   /* wh_format */
    uint32_t rate; /* bits per value, WH_FMT_ZFP_FIXED_RATE only; the GPU
                      decoder supports even rates 2..32 */
} wh_matrix_desc;

typedef struct wh_ctx wh_ctx;
typedef uint64_t wh_mat; /* matrix handle, never 0 */

#define WH_HOST 0   /* bytes are host memory: copied, the library owns it   */
#define WH_DEVICE 1 /* bytes are device memory: borrowed, the caller keeps it
                       alive and unchanged until wh_unload                   */

/* GEMV flags (accumulation of the cross-block row sums, Sec. 4.4). */
#define WH_ACC_DEFAULT 0u
#define WH_ACC_FP64 1u     /* FP32 block partial sums, FP64 accumulation    */
#define WH_ACC_TWOSUM 2u   /* FP32 block partial sums, compensated FP32
                              (TwoSum) accumulation                          */
#define WH_HOST_DIRECT 8u  /* wh_gemv_host only: the kernel reads the
                              page-locked stream over the link itself */
#define WH_PAPER_MP 4u     /* Fig. 7 exactly: every FP32 product added to an
                              FP64 sum; slowest; zfp and F32 formats only    */

/* Status text (static storage, never NULL). */
const char *wh_status_str(wh_status st);

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` bounds
 * the device memory the serving loop may hold for request buffers (0 = 1 GiB
 * default).  No GPU / bad device -> WH_ERR_DEVICE.  The environment
 * variables WH_GEMV_LANES (4, 8, ..., 512 lanes per block row),
 * WH_GEMV_ROWS (1, 2 or 4 block rows per lane group) and WH_GEMV_SLABS
 * (column slabs), read here, fix the compressed GEMV's launch shape instead
 * of the planner's choice, and WH_MRHS_SLABS the multi-RHS kernel's column
 * slabs (for launch-shape sweeps); invalid values are ignored.  Results stay within the stated tolerances for every shape.
 * WH_MRHS_FP32=1 keeps FP32 right-hand sides on the 16x16x4 FP32 matrix-core
 * instruction for every k (by default up to 4 right-hand sides run on the
 * 4x4x1 one, and from 17 up the FP32 operands are each split into three
 * BF16 parts and their six significant products run on the BF16 matrix
 * cores; the result stays within the FP32 tolerance either way).
 * WH_SERVE_PACE (a number from 1 to 16, default 4) paces a served matrix
 * whose requests can no longer meet their deadlines: while other work waits,
 * it gets one launch per that many of its launch times.
 * WH_SERVE_MARGIN_US (default 1000) is the margin, in microseconds, that a
 * held request keeps before its deadline beyond its estimated pass.
 * WH_SERVE_CHUNK_VALUES (a positive integer, default 2^28) bounds the matrix
 * values one serving launch covers: the serving loop runs each pass over a
 * larger matrix as launches over consecutive row chunks, so that batches of
 * other matrices get the device between chunks.  WH_SERVE_SHED=F (an integer
 * 1..1000; unset or 0 = off) turns on load shedding: wh_submit rejects a
 * request with WH_ERR_BUDGET while its matrix's oldest queued request has
 * waited more than F of its own deadlines. */
wh_status wh_create(int hip_device, uint64_t hbm_budget_bytes, wh_ctx **out);

/* Destroy a context: waits for its work, frees what it owns. */
wh_status wh_destroy(wh_ctx *ctx);

/* Bytes a matrix of this description occupies (exact). */
wh_status wh_storage_bytes(const wh_matrix_desc *desc, uint64_t *nbytes);

/* Register a resident matrix (Sec. 2.1 field matrix; Sec. 4.3 offline
 * encoding).  `nbytes` must equal wh_storage_bytes(desc).  where = WH_HOST:
 * the bytes are copied to device memory the library owns (synchronously);
 * WH_DEVICE: the device buffer is borrowed. */
wh_status wh_load_compressed(wh_ctx *ctx, const wh_matrix_desc *desc, const void *bytes, uint64_t nbytes,
                             int where, wh_mat *out);

/* Forget a matrix (frees library-owned memory after pending work).  If the
 * serving loop holds the matrix, its batches in flight finish first (and
 * are delivered); its requests not yet started complete with
 * WH_ERR_NOT_FOUND, and its slots return to the HBM budget. */
wh_status wh_unload(wh_ctx *ctx, wh_mat m);

/* y[i - row_begin] = sum_j M[i, j] u[j] for rows [row_begin, row_end)
 * (Eq. 2 / Eq. 5 over the slit rows of a resident field matrix, Fig. 2).
 * d_u: cols FP32; d_y: (row_end - row_begin) FP32.  Any range with
 * row_begin <= row_end <= rows (else WH_ERR_SHAPE), except that the
 * block-scaled FP8 format needs both ends on multiples of 4.  The compressed
 * format decodes the range's first and last block rows whole and writes only
 * the range's rows.  d_u 16-byte aligned.
 *
 * Compressed formats are decoded inside the kernel, never written out.  A
 * block's contribution is taken in coefficient space: its coefficients,
 * scaled by the block exponent, times B^T u (B = the inverse transform's
 * linear part), in FP32; B is applied to each row group's sums.  This equals
 * the product with the decoded matrix up to the transform's floor halvings
 * (a few units of each block's last bit: ~1e-8 relative) for streams an
 * encoder produced.  Precondition: a compressed matrix's stream is encoder
 * output (wh_encode, wh_encode_var, or any encoder of the same format).  On
 * other bytes the call still runs and stays in bounds, but y is then only
 * some function of the bytes, not the product with what wh_decode returns
 * for them; wh_decode is defined on every byte string.  Row sums are FP64
 * (default) or compensated FP32 across
 * blocks; y is rounded once to FP32 (Fig. 7).  WH_PAPER_MP instead
 * multiplies every bit-exact decoded value by u in FP32 and adds each
 * product to an FP64 sum.  Dense formats multiply the stored values.
 *
 * Workspace: when the plan splits the columns into slabs (most large
 * compressed matrices, wh_gemv_plan_info), the FP64 slab partials live in a
 * workspace of the context's, grown (freed and reallocated) on demand.  Such
 * a call returns WH_ERR_INVALID while `stream` is being captured into a HIP
 * graph, since a later call could free the memory the graph would keep
 * using; wh_gemv_noalloc is the form to capture.  The same holds for
 * wh_gemv_batched and wh_gemv_host. */
wh_status wh_gemv(wh_ctx *ctx, wh_mat m, const float *d_u, float *d_y, uint32_t row_begin, uint32_t row_end,
                  uint32_t flags, void *stream);

/* wh_gemv without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc.  WHZ1 fixed-rate matrices only (else WH_ERR_FORMAT); arguments,
 * launch plan, kernels and result as wh_gemv, so y is the same.
 *
 * Workspace: the FP64 slab partials live in a device array of the library's
 * of WH_NOALLOC_SCRATCH_BYTES (64 MiB), one per GPU, held from the first
 * wh_create on that GPU until the process ends.  A call whose plan needs more
 * (column slabs x the range's rows rounded up to whole block rows x 8 bytes;
 * wh_gemv_plan_info gives both) returns WH_ERR_SCRATCH and launches nothing:
 * 65536 x 65536 needs 32 MiB, and no matrix of up to 2^33 values more than
 * 44 MiB.  Calls whose work overlaps on one GPU (other
 * streams, other contexts) share that array and race; calls in order on one
 * stream are safe.  The array keeps the last call's contents; nothing in it
 * has to start at zero.  No hipMalloc, hipFree, event or memset is issued, so
 * the call can be captured into a graph (the graph then keeps using the
 * array). */
#define WH_NOALLOC_SCRATCH_BYTES (64ull << 20)
wh_status wh_gemv_noalloc(wh_ctx *ctx, wh_mat m, const float *d_u, float *d_y, uint32_t row_begin,
                          uint32_t row_end, uint32_t flags, void *stream);

/* The launch shape the fused compressed GEMV would use for rows
 * [row_begin, row_end) of a rows x cols matrix at `rate` bits/value on a
 * device with num_cus CUs (diagnostics; no context, no GPU): out9 = {lanes
 * per block row, block rows per lane group, row tiles, column slabs, block
 * columns per slab, first block row, one past the last block row, rows of the
 * first block row before the range, lanes per workgroup}.  The workgroups
 * launched are row tiles x column slabs.  An unsupported rate ->
 * WH_ERR_INVALID. */
wh_status wh_gemv_plan_info(uint32_t rows, uint32_t cols, uint32_t row_begin, uint32_t row_end, int num_cus,
                            uint32_t rate, uint32_t *out9);

/* Y = M U for k right-hand sides.  The paper's GEMV takes one vector
 * (Sec. 4.4); several at once is this library's addition, for the serving
 * loop's batches.  d_U: k vectors of
 * cols values, vector r at d_U + r*ldu (ldu >= cols), dtype 0 = FP32,
 * 1 = BF16.  d_Y: k vectors of rows FP32 at d_Y + r*ldy (ldy >= rows).
 * 1 <= k <= 64.  zfp format only; WH_PAPER_MP only with k = 1.  The matrix
 * cores contract the scaled coefficients against B^T U (as wh_gemv), FP64
 * across columns.  FP32 U: on the FP32 matrix cores up to 16 right-hand
 * sides (4x4x1 MFMAs up to 4, 16x16x4 above); from 17 up each FP32 operand
 * is split into three BF16 parts and the six significant part products run
 * on the BF16 matrix cores (within the FP32 tolerance; WH_MRHS_FP32=1 at
 * wh_create keeps the 16x16x4 FP32 cores).  BF16 U:
 * both operands rounded to BF16. */
#define WH_U_F32 0
#define WH_U_BF16 1
wh_status wh_gemv_batched(wh_ctx *ctx, wh_mat m, const void *d_U, int u_dtype, uint32_t k, uint32_t ldu,
                          float *d_Y, uint32_t ldy, uint32_t flags, void *stream);

/* y[i - row_begin] = sum_j M[i, j] u[j] for rows [row_begin, row_end) of a
 * WHZ1 matrix that stays in HOST memory (Sec. 4.2: the model matrix lives
 * in host DDR and crosses PCIe compressed; Sec. 4.3, Table 1: the
 * transfers are pipelined with the work on the GPU).  h_code: the matrix's whole rate-`rate` stream (rows x
 * cols, layout as WH_FMT_ZFP_FIXED_RATE), host memory; only the block rows
 * of the range are read.  The block rows cross the link in chunks of
 * chunk_rows rows (a multiple of 4; 0 = about 32 MiB of code per chunk) on
 * a copy stream of the library's, into two device staging buffers used in
 * turn; each chunk's fused decode + GEMV runs on `stream` once its copy has
 * landed, while the next chunk is in flight.  Copies overlap the GPU's work
 * only from page-locked memory (hipHostMalloc, torch pin_memory); pageable
 * memory works but its copies are staged by the runtime.  With
 * WH_HOST_DIRECT in flags there is no copy: the fused kernel reads the
 * page-locked stream over the link itself (pageable memory ->
 * WH_ERR_INVALID).  h_code must stay valid and unchanged until the work on
 * `stream` has finished.  d_u, d_y, other flags, ranges and errors as
 * wh_gemv; the staging buffers belong to the context (grown on demand, freed
 * by wh_destroy). */
wh_status wh_gemv_host(wh_ctx *ctx, const void *h_code, uint32_t rows, uint32_t cols, uint32_t rate,
                       const float *d_u, float *d_y, uint32_t row_begin, uint32_t row_end, uint32_t chunk_rows,
                       uint32_t flags, void *stream);

/* Page-locked host memory for h_code of wh_gemv_host (hipHostMalloc): the
 * copies of such memory overlap the GPU's work.  Needs no context.  Freed by
 * wh_host_free (NULL is a no-op) once no queued work reads it. */
wh_status wh_host_alloc(uint64_t bytes, void **h_ptr);
wh_status wh_host_free(void *h_ptr);

/* Variable-rate encoder (host; the paper encodes offline, Sec. 4.3): h_M
 * rows x cols FP32 row-major in host memory -> h_out (cap bytes of host
 * memory), the storage of format fmt (WH_FMT_ZFP_FIXED_PRECISION or
 * _ACCURACY) with parameter `rate` as in wh_matrix_desc; *out_bytes = the
 * bytes written (pass them to wh_load_compressed).  cap >=
 * wh_var_capacity_bytes(rows, cols) always suffices.  NaN/Inf ->
 * WH_ERR_INVALID.  Needs no context.  wh_gemv (not WH_PAPER_MP) and
 * wh_decode take these formats; wh_gemv_batched and the serving loop do
 * not (WH_ERR_FORMAT). */
uint64_t wh_var_index_bytes(uint32_t rows, uint32_t cols);
uint64_t wh_var_capacity_bytes(uint32_t rows, uint32_t cols);
wh_status wh_encode_var(const float *h_M, uint32_t rows, uint32_t cols, int32_t fmt, uint32_t rate, void *h_out,
                        uint64_t cap, uint64_t *out_bytes);

/* The thermal step (Sec. 2.1, Eq. 1): d_T_next = A d_T + B d_u, for n
 * temperatures.  A is n x n in CSR: d_row_ptr[n + 1] (d_row_ptr[0] = 0,
 * nondecreasing, d_row_ptr[n] = nnz), d_col[nnz] (column of each entry, < n),
 * d_val[nnz] FP32; B is diagonal, d_b[n] FP32.  d_T, d_u, d_T_next: n FP32;
 * d_T_next must not be d_T.  Each row is summed in FP64 and rounded once to
 * FP32.  Entries past nnz and columns >= n are skipped (wrong values, never a
 * stray access).  All device memory, owned by the caller. */
wh_status wh_thermal_step(wh_ctx *ctx, uint32_t n, uint32_t nnz, const uint32_t *d_row_ptr, const uint32_t *d_col,
                          const float *d_val, const float *d_b, const float *d_T, const float *d_u, float *d_T_next,
                          void *stream);

/* `steps` thermal steps in a row: T_{k+1} = A T_k + B u_k for k = 0 ..
 * steps - 1, with u_k = d_U + k * ldu (ldu >= n).  d_T holds T_0 on entry
 * and T_steps when the work on `stream` is done; d_work (n FP32, not d_T) is
 * the other half of the ping-pong.  Arguments otherwise as wh_thermal_step. */
wh_status wh_thermal_run(wh_ctx *ctx, uint32_t n, uint32_t nnz, const uint32_t *d_row_ptr, const uint32_t *d_col,
                         const float *d_val, const float *d_b, float *d_T, const float *d_U, uint64_t ldu,
                         uint32_t steps, float *d_work, void *stream);

/* Bit-exactness probe: decode blocks [block_begin, block_begin + nblocks)
 * of a zfp matrix into d_out[nblocks][16] FP32 (v = 4r + c in a block;
 * partial blocks come out with their edge padding). */
wh_status wh_decode_debug(wh_ctx *ctx, wh_mat m, uint64_t block_begin, uint64_t nblocks, float *d_out,
                          void *stream);

/* Decode a whole zfp matrix into a dense row-major FP32 matrix d_out
 * (rows x cols; the edge padding is dropped) -- the "decode, then GEMV"
 * path of Fig. 11. */
wh_status wh_decode(wh_ctx *ctx, wh_mat m, float *d_out, void *stream);

/* Offline encoder (Sec. 4.3: encoding happens before the loop starts), run
 * on the GPU: WHZ1 fixed-rate code of the dense FP32 matrix d_M (rows x
 * cols, row-major, any rows, cols >= 1, 16-byte aligned) into d_stream
 * (wh_storage_bytes bytes; every byte is written).  NaN/Inf values encode as zero blocks and are counted in
 * *d_bad (device uint32, may be NULL; not cleared by the call). */
wh_status wh_encode(wh_ctx *ctx, const float *d_M, uint32_t rows, uint32_t cols, uint32_t rate, void *d_stream,
                    uint32_t *d_bad, void *stream);

/* Quantise a dense FP32 matrix into a reduced-precision storage format
 * (WH_FMT_F16 / BF16 / FP8E4M3_BS4); d_out holds wh_storage_bytes. */
wh_status wh_quantize(wh_ctx *ctx, const float *d_M, uint32_t rows, uint32_t cols, int32_t fmt, void *d_out,
                      void *stream);

/* Diagnostics: the device's read-only streaming ceiling.  Reads the nbytes
 * of d_buf (16-byte aligned, nbytes a multiple of 16) once with 16-byte
 * non-temporal loads and XORs every 32-bit word of it into *d_out (device
 * uint32, not cleared by the call: clear it first to get the buffer's XOR).
 * The time of this call is the HBM read rate a kernel that only streams its
 * input can reach -- the practical ceiling for the compressed GEMV, which
 * reads its stream once and writes almost nothing (the paper prices its
 * kernels against memory bandwidth, Sec. 4.1, Fig. 4). */
wh_status wh_stream_read(wh_ctx *ctx, const void *d_buf, uint64_t nbytes, uint32_t *d_out, void *stream);

/* ------------------------------------------------------------------ */
/* Serving loop (Sec. 1: firm deadlines; Fig. 2: per-millisecond calls) */
/* ------------------------------------------------------------------ */
typedef struct {
    wh_mat mat;          /* target resident matrix                         */
    const float *U;      /* k dose vectors of cols FP32, contiguous         */
    int u_on_device;     /* 0: U is host memory (staged by the library)    */
    uint32_t k;          /* 1..8 right-hand sides                           */
    float *Y;            /* k x rows FP32 result                            */
    int y_on_device;     /* 0: Y is host memory (copied back)               */
    uint64_t deadline_ns;/* relative deadline from arrival                  */
    uint64_t arrival_ns; /* 0 = stamp on submit (CLOCK_MONOTONIC ns)        */
} wh_request;

typedef struct {
    wh_status status;    /* WH_PENDING, WH_OK or an error                   */
    uint64_t t_arrive_ns, t_start_ns, t_done_ns;
    int32_t missed;      /* 1 if t_done > arrival + deadline (still valid)  */
    uint32_t batch_size; /* requests in the launch that served this one     */
} wh_result;

/* Enqueue a request; returns a ticket.  Thread-safe, never blocks on the GPU.
 * The first request for a matrix sets up its serving state: one device slot
 * of 64 right-hand sides (U, Y and FP64 slab partials, charged to the
 * context's HBM budget) with one captured hipGraph per k-bucket; a second
 * slot is added later if a batch has to wait and the budget has room.  Rejected at
 * once with WH_ERR_BUDGET if not even one slot of that matrix fits the
 * budget, if k > 64, or (load shedding, see wh_create) while the matrix's
 * queue is too far behind.  U and Y must stay valid until wh_poll reports
 * the request done.  zfp matrices only. */
wh_status wh_submit(wh_ctx *ctx, const wh_request *req, uint64_t *ticket);

/* Non-blocking: WH_PENDING until the request's result is in Y, then WH_OK
 * (result filled; the ticket is then retired) or the request's error. */
wh_status wh_poll(wh_ctx *ctx, uint64_t ticket, wh_result *out);

#ifdef __cplusplus
}
#endif

#endif /* WH_H_ */
