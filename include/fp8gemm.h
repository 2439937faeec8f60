/*
 * fp8gemm.h - C ABI of the MI355X (gfx950) FP8 GEMM library, libfp8gemm.so.
 *
 * The operation (arXiv 2602.10262): FP8 x FP8 matrix products with FP32
 * accumulation (Sec. 2, "FP8 Matrix Cores"), dense and with 2:4 structured
 * sparsity along the reduction dimension (Sec. 2, "Structured Sparsity";
 * Sec. 7), with the sparse encoding as a step of its own ahead of the product
 * (Sec. 7.1.1, where the encoding cost is measured apart from the GEMM),
 * independent GEMMs running concurrently on separate HIP streams (Sec. 6,
 * Sec. 8.2), and transformer-style sequences of many GEMMs (Sec. 8.1).
 *
 * Conventions (every entry point):
 *   - Plain C.  Every call returns fp8_status; fp8_last_error() returns a
 *     thread-local text for the last failure of the calling thread.
 *   - Tensor pointers are DEVICE pointers owned by the caller; the library
 *     never frees them and keeps no reference after the call's stream work.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Kernel calls are asynchronous on it and never synchronise the host.
 *   - FP8 formats are the OCP ones (E4M3: bias 7, max 448, no infinity;
 *     E5M2: bias 15, max 57344, IEEE infinities).
 *   - Shapes: M, N, K >= 1 (else FP8_ERR_SHAPE).  Leading dimensions are in
 *     elements and at least the row length.  FP8 operand base pointers and
 *     leading dimensions must be multiples of 16 bytes (else FP8_ERR_ALIGN).
 *   - Argument checking is done on the host before any launch: a call that
 *     returns an error has enqueued nothing.
 */
#ifndef FP8GEMM_H
#define FP8GEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FP8_OK = 0,
    FP8_ERR_ARG = 1,          /* null or inconsistent argument, workspace too small */
    FP8_ERR_SHAPE = 2,        /* a dimension out of range */
    FP8_ERR_ALIGN = 3,        /* pointer or leading dimension not 16-byte aligned */
    FP8_ERR_UNSUPPORTED = 4,  /* valid request the library has no kernel for */
    FP8_ERR_HIP = 5,          /* a HIP runtime call failed (text in fp8_last_error) */
    FP8_ERR_NOMEM = 6,        /* a library-owned allocation failed */
    FP8_ERR_BUDGET = 7,       /* server: request larger than the whole HBM budget */
    FP8_ERR_CLOSED = 8,       /* server: shutting down */
    FP8_ERR_PENDING = 9,      /* server: ticket not finished yet */
    FP8_ERR_TIMEOUT = 10      /* server: wait timed out */
} fp8_status;

typedef enum { FP8_E4M3 = 0, FP8_E5M2 = 1 } fp8_fmt;
/* Output types (BF16 and FP16 rounded to nearest even). */
typedef enum { FP8_OUT_F32 = 0, FP8_OUT_BF16 = 1, FP8_OUT_F16 = 2 } fp8_out;
/* TENSOR: one scale.  ROW: one per row of A (M values) / per column of B (N values). */
typedef enum { FP8_SCALE_TENSOR = 0, FP8_SCALE_ROW = 1 } fp8_scale_kind;
/* Which operand is 2:4-compressed.  A: the M x K activations; B: the weight,
 * stored as its N x K transpose (one compressed row per output column). */
typedef enum { FP8_SPARSE_A = 0, FP8_SPARSE_B = 1 } fp8_sparse_side;

const char *fp8_last_error(void);
int fp8_version(void);

/* ------------------------------------------------------------------------ */
/* Quantization: amax -> scale -> FP8 codes.                                 */
/* ------------------------------------------------------------------------ */
/* The per-tensor / per-row scaling that brings FP32 data into the FP8 range
 * (the amax and scale reductions of the method).  For each tensor (kind =
 * TENSOR) or each row (kind = ROW) of the row-major rows x cols FP32 matrix x:
 *   amax = max |x|  (NaN if any element is NaN)
 *   s = fl32(fmax / amax), d = fl32(1 / s)   (IEEE divisions; fmax = 448 for
 *       E4M3, 57344 for E5M2); when amax is 0 or not finite, or s or d is 0
 *       or not finite, s = d = 1
 *   q = encode(fl32(x * s)): round to nearest even, saturating to +-fmax,
 *       NaN -> 0x7F | sign, -0 kept.
 * Outputs: q (row-major, ldq), scale = s and descale = d (1 or rows floats).
 * ws: device workspace of fp8_quantize_workspace_size() bytes (4 bytes for
 * TENSOR, 0 for ROW); its content need not be initialised.
 * Requirements: x 16-byte aligned with ldx % 4 == 0, q aligned with
 * ldq % 16 == 0. */
fp8_status fp8_quantize_workspace_size(int64_t rows, int64_t cols, fp8_scale_kind kind, size_t *bytes);
fp8_status fp8_quantize(const float *x, int64_t rows, int64_t cols, int64_t ldx, fp8_fmt fmt,
                        fp8_scale_kind kind, uint8_t *q, int64_t ldq, float *scale, float *descale,
                        void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Dense GEMM.                                                               */
/* ------------------------------------------------------------------------ */
/* C = diag(d_a) * (dec(A) x dec(B)) * diag(d_b), accumulated in FP32 from
 * exact FP8 products (Sec. 2: FP8 operands, FP32 accumulation), then
 * C[i,j] = (acc[i,j] * d_a[i]) * d_b[j] in FP32, stored as FP32 or as BF16
 * rounded to nearest even.
 *   a: row-major M x K codes, leading dimension lda (bytes)
 *   b: column-major K x N codes, i.e. N rows of K codes, leading dimension ldb
 *   a_descale: 1 float (TENSOR) or M floats (ROW); b_descale: 1 or N floats
 *   c: row-major M x N, leading dimension ldc (elements) */
typedef struct {
    int64_t M, N, K;
    const uint8_t *a; fp8_fmt a_fmt; int64_t lda;
    const uint8_t *b; fp8_fmt b_fmt; int64_t ldb;
    const float *a_descale; fp8_scale_kind a_kind;
    const float *b_descale; fp8_scale_kind b_kind;
    void *c; fp8_out c_type; int64_t ldc;
} fp8_gemm_args;

/* Kernel choice: tile is an index into the table fp8_tile_info() describes
 * (-1 = let the library choose: tuning cache, else heuristic); split_k >= 1
 * splits the reduction into that many fixed-order partial sums (0 = choose). */
typedef struct {
    int tile;
    int split_k;
} fp8_plan;

/* Describes compiled tile `tile`: macro-tile rows/cols, waves per workgroup,
 * whether it has a 2:4 kernel (*sparse) and a dense kernel (*dense) - a plan
 * naming a tile without the kernel it needs is rejected with FP8_ERR_ARG -
 * and whether it is an exact-sum tile (*exact: the FP8 codes are decoded to
 * BF16 and summed on the BF16 MFMA, whose error stays inside the bound
 * 4 K 2^-24 sum |a b| for every K; the FP8 MFMA tiles guarantee that bound
 * only for K >= 3584, so plans the library chooses use exact-sum tiles below
 * that K).  The exact-sum tiles that stage FP8 codes through the LDS-DMA
 * ring need K to be a multiple of 16 (128 with a 2:4 operand); a plan naming
 * one for any other K runs on the register-staged exact-sum tile 27.  Any out
 * pointer may be NULL.  FP8_ERR_ARG past the last tile. */
fp8_status fp8_tile_info(int tile, int *block_m, int *block_n, int *waves, int *sparse, int *dense,
                         int *exact);
int fp8_num_tiles(void);

/* The plan the library would use for these arguments (NULL plan = choose). */
fp8_status fp8_gemm_plan_resolve(const fp8_gemm_args *args, const fp8_plan *plan, fp8_plan *resolved);
fp8_status fp8_gemm_workspace_size(const fp8_gemm_args *args, const fp8_plan *plan, size_t *bytes);
/* ws may be NULL when the workspace size is 0. */
fp8_status fp8_gemm(const fp8_gemm_args *args, const fp8_plan *plan, void *ws, size_t ws_bytes,
                    void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): fp8_gemm
 * with the same arguments, plan choice and kernels, whose split-K partial
 * sums live in a fixed device array of the library (fp8_noalloc_scratch_bytes()
 * bytes per GPU, 32 MiB, held from the first call on a GPU until the process
 * ends) instead of a workspace.  It calls no allocator.  A plan whose partial
 * sums exceed that size is refused with FP8_ERR_UNSUPPORTED before anything is
 * enqueued.  All calls on one GPU share that GPU's array: calls that overlap
 * in time on one GPU race and must be ordered by the caller (one stream, or
 * events).  Results equal fp8_gemm's with the same plan bit for bit. */
size_t fp8_noalloc_scratch_bytes(void);
fp8_status fp8_gemm_noalloc(const fp8_gemm_args *args, const fp8_plan *plan, void *stream);

/* ------------------------------------------------------------------------ */
/* 2:4 structured sparsity.                                                  */
/* ------------------------------------------------------------------------ */
/* Prunes a row-major rows x K code matrix to 2:4 along K (Sec. 2 and Sec. 7:
 * two of every four consecutive elements become zero) and compresses it.
 * In each group of four (k = 4g .. 4g+3) the two elements of largest
 * magnitude survive, equal magnitudes going to the lower index; magnitude is
 * compared on the 7-bit field code & 0x7F, which orders every finite code by
 * |value| and ranks NaN/infinity codes above all finite ones.
 *   values[r*ldv + 2g + t]: survivor t (t = 0, 1) in ascending index order
 *   meta[r*ldm + g/2]: nibble g % 2 (low nibble = even g) = i0 | i1 << 2 with
 *                      i0 < i1 the survivor positions; the little-endian
 *                      32-bit word w of a row describes groups 8w .. 8w+7
 *   mask[r*ldm + k/8]: bit k % 8 set iff element k survives (mask may be NULL)
 * ldv = K/2 and ldm = K/8 (the compressed rows are packed).  K % 8 == 0 and
 * the x/values/meta base pointers 16-byte aligned are required. */
fp8_status fp8_sparse24_prune_compress(const uint8_t *x, fp8_fmt fmt, int64_t rows, int64_t K,
                                       int64_t ldx, uint8_t *values, uint8_t *meta, uint8_t *mask,
                                       void *stream);
/* Quantize and prune in one pass (the encode step of the 2:4 path, Sec. 7.1.1,
 * whose cost the method measures separately from the GEMM): the FP32 rows x K
 * matrix x is quantized exactly as fp8_quantize does (same amax, scale and
 * codes, per tensor or per row) and the codes are pruned and compressed
 * exactly as fp8_sparse24_prune_compress does, without the dense codes ever
 * being written.  Outputs: values, meta, mask (may be NULL) in the layout
 * above; scale and descale (1 or rows floats).  ws: fp8_quantize_workspace_size
 * (rows, K, kind) bytes (4 for TENSOR, none for ROW).  Requirements: K % 8 ==
 * 0, x 16-byte aligned with ldx % 4 == 0, values/meta/mask 16-byte aligned.
 * Errors: FP8_ERR_ARG (null pointer, bad enum, ldx < K, workspace),
 * FP8_ERR_SHAPE, FP8_ERR_ALIGN; nothing is enqueued on error. */
fp8_status fp8_quantize_prune24(const float *x, int64_t rows, int64_t K, int64_t ldx, fp8_fmt fmt,
                                fp8_scale_kind kind, uint8_t *values, uint8_t *meta, uint8_t *mask,
                                float *scale, float *descale, void *ws, size_t ws_bytes, void *stream);

/* The pruned dense matrix: out[r*ldo + k] = survivor code or +0 (0x00). */
fp8_status fp8_sparse24_decompress(const uint8_t *values, const uint8_t *meta, int64_t rows,
                                   int64_t K, uint8_t *out, int64_t ldo, void *stream);

/* C = A' x B with one operand given in the compressed form above.
 *   side A: (values, meta) hold the compressed M x K activations; g.a unused.
 *   side B: (values, meta) hold the compressed N x K transpose of B (a weight
 *           in its natural N x K layout); g.b unused.
 * Scales, formats and output as in fp8_gemm.  K % 128 == 0 is not required,
 * K % 8 == 0 is.  The result equals fp8_gemm on the decompressed operand up
 * to FP32 summation order. */
typedef struct {
    fp8_gemm_args g;
    fp8_sparse_side side;
    const uint8_t *values;
    const uint8_t *meta;
} fp8_sparse24_gemm_args;

fp8_status fp8_sparse24_gemm_workspace_size(const fp8_sparse24_gemm_args *args, const fp8_plan *plan,
                                            size_t *bytes);
fp8_status fp8_sparse24_gemm(const fp8_sparse24_gemm_args *args, const fp8_plan *plan, void *ws,
                             size_t ws_bytes, void *stream);

/* Both operands 2:4-compressed (the both-side sparsity pattern, Sec. 7.1):
 * C = A' x W'^T, where A' (M x K activations) and W' (N x K weight rows) are
 * the pruned matrices given in the compressed form above, i.e. the sum runs
 * over the k that both operands keep.  g.a and g.b are unused; formats,
 * scales and output as in fp8_gemm.  No instruction takes two compressed
 * operands: one operand feeds the 2:4 MFMA and the other is expanded to its
 * dense rows inside the kernel (never in memory), so it is read from HBM at
 * 0.625 bytes per element.  Plans: tiles 0, 3, 11, 12 (FP8 MFMA) and the
 * exact-sum tiles 25, 26, 27 (chosen for K < 3584, as for the other GEMMs); any
 * other tile is rejected with FP8_ERR_ARG.  Requirements: K % 8 == 0 and the
 * four compressed pointers 16-byte aligned.  The result equals fp8_gemm on
 * the two decompressed operands up to FP32 summation order. */
typedef struct {
    fp8_gemm_args g;
    const uint8_t *a_values, *a_meta;   /* compressed M x K activations */
    const uint8_t *b_values, *b_meta;   /* compressed N x K weight rows */
} fp8_sparse24_both_gemm_args;

fp8_status fp8_sparse24_both_gemm_plan_resolve(const fp8_sparse24_both_gemm_args *args, const fp8_plan *plan,
                                               fp8_plan *resolved);
fp8_status fp8_sparse24_both_gemm_workspace_size(const fp8_sparse24_both_gemm_args *args, const fp8_plan *plan,
                                                 size_t *bytes);
fp8_status fp8_sparse24_both_gemm(const fp8_sparse24_both_gemm_args *args, const fp8_plan *plan, void *ws,
                                  size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Higher-precision GEMMs (the FP32 and 16-bit stages of Sec. 8.3).          */
/* ------------------------------------------------------------------------ */
/* The mixed-precision sequence of Sec. 8.3 runs FP32 and 16-bit matrix
 * operations beside the FP8 ones.  C = diag(s_a) (A x B) diag(s_b) with
 *   a: row-major M x K, b: N rows of K (column-major K x N), both of type
 *      ab_type (FP32 on the FP32 MFMA, FP16 / BF16 on the 16-bit MFMA with
 *      exact products and FP32 sums); lda, ldb, ldc count elements
 *   a_scale: 1 or M floats, b_scale: 1 or N floats (device)
 *   c: row-major M x N, FP32, BF16 or FP16 (RNE), computed as
 *      (acc * s_a[i]) * s_b[j] in FP32.
 * The result is within 4 K 2^-24 sum |a b s_a s_b| of the exact one (plus the
 * output rounding).  Requirements: K <= 2^20, a and b 16-byte aligned with
 * 16-byte row strides.  Errors: FP8_ERR_ARG, FP8_ERR_SHAPE, FP8_ERR_ALIGN;
 * nothing is enqueued on error.  Asynchronous on `stream`. */
typedef enum { FP8_HP_F32 = 0, FP8_HP_F16 = 1, FP8_HP_BF16 = 2 } fp8_hp_type;
typedef struct {
    int64_t M, N, K;
    const void *a; int64_t lda;
    const void *b; int64_t ldb;
    fp8_hp_type ab_type;
    const float *a_scale; fp8_scale_kind a_kind;
    const float *b_scale; fp8_scale_kind b_kind;
    void *c; fp8_out c_type; int64_t ldc;
    int tile_rows;            /* 0 = choose; 64, 128 or 256 (square tiles) */
} fp8_hp_gemm_args;
fp8_status fp8_hp_gemm(const fp8_hp_gemm_args *args, void *stream);

/* ------------------------------------------------------------------------ */
/* Mixed-precision sequences and their co-scheduling (Sec. 8.3, Sec. 9.2).   */
/* ------------------------------------------------------------------------ */
/* The mixed-precision workload of Sec. 8.3 is a sequence of matrix
 * operations in different precisions; Sec. 9.2 advises co-scheduling
 * kernels of similar wavefront needs and co-locating memory-bound FP8 work
 * with compute-bound FP32 work.  A chain is a sequence of GEMM stages
 * Y_s = X_s W_s^T over M rows, stage s in its own precision; its K is the
 * previous stage's N (stage 0: in_width).  Stage s writes its result in the
 * input type of stage s + 1 (FP32, FP16 or BF16, rounded to nearest even by
 * the GEMM epilogue; FP32 for an FP8 stage, which quantizes its input per
 * row to E4M3 with fp8_quantize before its fp8_gemm).  The last stage writes
 * FP32.  n_chains independent chains share the weights.
 *   w: N x K weight rows in the stage's type, leading dimension K, 16-byte
 *      aligned (FP8: E4M3 codes)
 *   w_scale: FP8 stage: N descales (or NULL = 1); other stages: NULL = 1, or
 *            N column scales
 * Stage widths must give 16-byte rows (K a multiple of 16 for FP8 stages).
 * fp8_chain_create allocates every activation buffer, the FP8 staging and
 * split-K workspace of each chain, max_streams (1..8) streams of default
 * priority and the timing events; fp8_chain_destroy frees them (after
 * draining).  fp8_chain_buffer gives stage s's input buffer of a chain
 * (row-major M x K_s, leading dimension *ld elements; stage = n_stages gives
 * the FP32 output) - the caller fills stage 0's input before fp8_chain_run.
 * fp8_chain_run synchronizes the device, enqueues every chain under the
 * schedule and waits for the end:
 *   SERIAL    one stream, chain after chain;
 *   IN_PHASE  chain c on stream c % n_streams, all streams starting together
 *             (the stages that overlap share a precision);
 *   STAGGERED as IN_PHASE, but stream k starts once stream k - 1 has finished
 *             its first stage (neighbouring streams overlap different
 *             precisions).
 * Results do not depend on the schedule (same kernels and plans).  Stats:
 * makespan, per-precision mean and coefficient of variation of the stage
 * times (each stage bracketed by events on its stream: the span its kernels
 * took, contention included; an FP8 stage includes its quantize) and
 * aggregate TFLOP/s (2 M N K per stage).  fp8_chain_stage_ms gives one
 * stage's time of the last run. */
typedef enum { FP8_STAGE_F32 = 0, FP8_STAGE_F16 = 1, FP8_STAGE_BF16 = 2, FP8_STAGE_FP8 = 3 } fp8_stage_prec;
typedef enum { FP8_CHAIN_SERIAL = 0, FP8_CHAIN_IN_PHASE = 1, FP8_CHAIN_STAGGERED = 2 } fp8_chain_schedule;
typedef struct {
    int precision;            /* fp8_stage_prec */
    int64_t N;
    const void *w;
    const float *w_scale;
} fp8_chain_stage;
typedef struct {
    double makespan_ms;
    double stage_ms_mean[4];  /* indexed by fp8_stage_prec */
    double stage_ms_cv[4];
    int stage_count[4];
    double tflops;
} fp8_chain_stats;
typedef struct fp8_chain fp8_chain;
fp8_status fp8_chain_create(const fp8_chain_stage *stages, int n_stages, int64_t M, int64_t in_width, int n_chains,
                            int max_streams, fp8_chain **out);
fp8_status fp8_chain_buffer(fp8_chain *chain, int chain_index, int stage, void **ptr, int64_t *ld);
fp8_status fp8_chain_run(fp8_chain *chain, int schedule, int n_streams, fp8_chain_stats *stats);
fp8_status fp8_chain_stage_ms(fp8_chain *chain, int chain_index, int stage, double *ms);
fp8_status fp8_chain_destroy(fp8_chain *chain);

/* ------------------------------------------------------------------------ */
/* Autotuner.                                                                */
/* ------------------------------------------------------------------------ */
/* Times every (tile, split_k) candidate for these arguments on `stream` with
 * HIP events (two warm-up calls, then iters timed calls, median taken),
 * records the best in the in-process tuning cache and returns it.  The
 * caller's c buffer is overwritten.  Workspace for the largest candidate is
 * allocated by the library for the duration of the call.  Candidates are the
 * exact-sum tiles when K < 3584 and the FP8 MFMA tiles otherwise (see
 * fp8_tile_info).  Keyed on (M and N rounded up to powers of two, K,
 * formats, output type, scale kinds, dense or sparse side). */
fp8_status fp8_tune_gemm(const fp8_gemm_args *args, int iters, void *stream, fp8_plan *best,
                         double *best_us);
fp8_status fp8_tune_sparse24_gemm(const fp8_sparse24_gemm_args *args, int iters, void *stream,
                                  fp8_plan *best, double *best_us);

/* Dense versus 2:4 on one product (Sec. 7.1, where the 2:4 path is measured
 * against dense on the same shapes to find where sparsity pays): both are
 * tuned as above and the record {shape, side, formats, output type, best
 * dense and 2:4 plans and times, use_sparse = 2:4 faster} is kept in the
 * tuning cache.  `sparse` and `dense` must describe the same M, N, K,
 * formats and output type; `dense` normally multiplies the decompressed
 * (pruned) operand, so both compute the same result.  Lookups round M up to
 * a power of two (N and K exact). */
typedef struct {
    int64_t M, N, K;
    int side;                 /* fp8_sparse_side of the 2:4 operand */
    int a_fmt, b_fmt, c_type;
    double dense_us, sparse_us;
    fp8_plan dense_plan, sparse_plan;
    int use_sparse;
} fp8_breakeven;
fp8_status fp8_tune_sparse_vs_dense(const fp8_sparse24_gemm_args *sparse, const fp8_gemm_args *dense,
                                    int iters, void *stream, fp8_breakeven *out);
/* *found = 1 and *out filled when a record covers the shape, else *found = 0. */
fp8_status fp8_tune_breakeven_lookup(int64_t M, int64_t N, int64_t K, fp8_sparse_side side, fp8_fmt a_fmt,
                                     fp8_fmt b_fmt, fp8_out c_type, fp8_breakeven *out, int *found);
int fp8_tune_breakeven_count(void);
fp8_status fp8_tune_breakeven_get(int index, fp8_breakeven *out);

/* Persist / restore the tuning cache (plans and dense-vs-2:4 records) as JSON
 * lines.  Every line carries the device ("<architecture> <product name>") and
 * HIP runtime version it was measured with; fp8_tune_cache_load skips lines
 * of another device or runtime, and lines it cannot parse.
 * fp8_tune_device_key gives the current device's identity ("none" and 0
 * without a device; buf may be NULL). */
fp8_status fp8_tune_cache_save(const char *path);
fp8_status fp8_tune_cache_load(const char *path);
void fp8_tune_cache_clear(void);
fp8_status fp8_tune_device_key(char *buf, size_t bytes, int *runtime_version);

/* ------------------------------------------------------------------------ */
/* Grouped GEMM: many independent problems in one persistent launch.         */
/* ------------------------------------------------------------------------ */
/* The batched form of the transformer-style sequence of FP8 GEMMs (Sec. 8.1):
 * every problem is a dense or 2:4 GEMM as above (FP32 accumulation, split_k 1)
 * and all of them run in one launch of a persistent kernel whose workgroups
 * take output tiles from a device work list ordered longest-first.
 * plan_create copies the problem descriptions to a device table (library
 * owned); the problems' device buffers must stay valid while the plan is
 * used.  tile: a tile index for every problem (-1 = library choice).
 * fp8_grouped_gemm enqueues the work on `stream`; it allocates nothing and
 * is capturable into a HIP graph.  With use_graph = 1 the first call captures
 * the launch into a graph and later calls replay it (same stream required). */
typedef struct {
    int is_sparse;
    fp8_gemm_args dense;            /* used when is_sparse == 0 */
    fp8_sparse24_gemm_args sparse;  /* used when is_sparse == 1 */
} fp8_group_problem;

typedef struct fp8_grouped_plan fp8_grouped_plan;
fp8_status fp8_grouped_plan_create(const fp8_group_problem *problems, int count, int tile,
                                   int use_graph, fp8_grouped_plan **plan);
fp8_status fp8_grouped_gemm(fp8_grouped_plan *plan, void *stream);
fp8_status fp8_grouped_plan_info(const fp8_grouped_plan *plan, int *tile, int64_t *num_tiles,
                                 int *num_workgroups);
fp8_status fp8_grouped_plan_destroy(fp8_grouped_plan *plan);
/* Times one grouped launch of `problems` with each tile the grouped kernel is
 * built for (plans created and destroyed inside; two warm-up launches, then
 * iters timed launches, median) and returns the fastest tile and its time.
 * The problems' outputs are overwritten.  Pass *best_tile to
 * fp8_grouped_plan_create. */
fp8_status fp8_grouped_tune(const fp8_group_problem *problems, int count, int iters, void *stream,
                            int *best_tile, double *best_us);

/* ------------------------------------------------------------------------ */
/* Serving: a continuous-batching request loop over several HIP streams.     */
/* ------------------------------------------------------------------------ */
/* Independent GEMM requests issued concurrently on separate streams (the
 * single-GPU analogue of the paper's concurrent-stream study, Sec. 6 and
 * Sec. 8.2).  Each request multiplies FP32 activations x (M x K, device,
 * quantized per token inside the server) by a registered FP8 weight (dense
 * or 2:4-compressed N x K rows with per-channel descales) into c (M x N).
 * A scheduler thread admits requests in arrival order while the transient
 * device memory they need (quantized activations, scales, workspace) fits in
 * hbm_budget_bytes and a stream slot is free, launches each on the least
 * loaded of num_streams streams, and retires it when its completion event
 * fires; requests that arrive meanwhile are admitted as memory and slots free
 * up.  The result of a request does not depend on what else is in flight.
 * Latency = completion - arrival, where arrival is the request's
 * arrival_time_s on the server clock (seconds since fp8_server_create) or,
 * when negative, the time of the submit call.
 * Ordering: the server runs on streams of its own that are not ordered
 * against the caller's streams, so x must hold its final values and c must
 * not be written by other pending work when fp8_server_submit is called
 * (synchronise the producing stream first); c is complete once wait/poll
 * report FP8_OK.
 * Failures: a request whose arguments the GEMM rejects fails with that
 * status before anything is enqueued; if a launch fails after part of the
 * request was enqueued, the ticket reports the failure only once that work
 * has finished, and its memory is reused only then. */
typedef struct {
    size_t hbm_budget_bytes;
    int num_streams;          /* 1 .. 16 */
    int max_inflight;         /* 0 = 4 * num_streams */
} fp8_server_config;

typedef struct {
    int64_t M;
    int weight_id;
    const float *x;           /* M x K FP32, row-major, ldx = K */
    void *c;                  /* M x N, row-major, ldc = N */
    fp8_out c_type;
    fp8_fmt x_fmt;            /* FP8 format the activations are quantized to */
    double arrival_time_s;
} fp8_request;

typedef struct {
    double p50_ms, p99_ms, mean_ms, max_ms;
    double tflops;            /* dense-equivalent 2*M*N*K over first arrival .. last completion */
    double span_s;
    double stream_cv;         /* coefficient of variation of per-stream busy time */
    double fairness_range;    /* 1 - (t_max - t_min) / t_mean over per-stream busy time */
    double fairness_minmax;   /* t_min / t_max over per-stream busy time */
    uint64_t done, failed, rejected, peak_inflight;
    size_t peak_bytes;
} fp8_server_stats;

typedef struct fp8_server fp8_server;
fp8_status fp8_server_create(const fp8_server_config *cfg, fp8_server **srv);
/* The same scheduler over a simulated executor, for testing admission and
 * statistics without a GPU: nothing is launched or read; a request occupies
 * its stream for launch_us + 2*M*N*K / (gflop_per_ms * 1e9) ms of wall time
 * and requests on one stream run one after another.  Weights and requests
 * may carry NULL device pointers.  Workspace needs are not modelled. */
fp8_status fp8_server_create_simulated(const fp8_server_config *cfg, double gflop_per_ms, double launch_us,
                                       fp8_server **srv);
/* Registers a weight: dense (meta NULL: w is N x K codes, K % 16 == 0) or 2:4
 * (w = values N x K/2, meta N x K/8, K % 8 == 0).  w_descale: N floats.
 * w and meta must be 16-byte aligned (FP8_ERR_ALIGN), shapes as stated
 * (FP8_ERR_SHAPE).  Buffers stay caller-owned. */
fp8_status fp8_server_register_weight(fp8_server *srv, const uint8_t *w, const uint8_t *meta,
                                      const float *w_descale, int64_t N, int64_t K, fp8_fmt fmt,
                                      int *weight_id);
/* Thread-safe, non-blocking.  FP8_ERR_BUDGET if the request alone exceeds the budget. */
fp8_status fp8_server_submit(fp8_server *srv, const fp8_request *req, uint64_t *ticket);
fp8_status fp8_server_poll(fp8_server *srv, uint64_t ticket);                 /* OK or PENDING */
fp8_status fp8_server_wait(fp8_server *srv, uint64_t ticket, int64_t timeout_us); /* <0: forever */
/* Latency of a finished ticket in milliseconds. */
fp8_status fp8_server_latency(fp8_server *srv, uint64_t ticket, double *ms);
fp8_status fp8_server_drain(fp8_server *srv);
fp8_status fp8_server_stats_get(fp8_server *srv, fp8_server_stats *stats);
fp8_status fp8_server_reset_stats(fp8_server *srv);
double fp8_server_now(fp8_server *srv);  /* seconds on the server clock */
fp8_status fp8_server_destroy(fp8_server *srv);                               /* drains first */

/* ------------------------------------------------------------------------ */
/* Microbenchmarks of the matrix cores and the LDS.                          */
/* ------------------------------------------------------------------------ */
/* The counterpart of the paper's FP8 MFMA characterisation (Sec. 5): one
 * workgroup per CU with waves_per_cu (1..16) wavefronts, each issuing
 * `chains` (1, 4 or 8) independent accumulator chains of one instruction for
 * `iters` rounds; *ms = device time of the launch.  kind: 0 = 16x16x128 FP8
 * MFMA, 1 = 32x32x64 FP8 MFMA, 2 = 16x16x128 FP8 2:4 SMFMAC, 3 = 32x32x64 FP8
 * SMFMAC.  With chains = 1 each instruction waits for the previous one
 * (dependent-issue latency); with more chains and waves the issue rate
 * (throughput).  A launch performs CUs x waves x 64 lanes worth of
 * chains x iters instructions; FLOPs per instruction: 2 M N K of the dense
 * shape (the SMFMAC counts the dense-equivalent 2 M N K).  Allocates a small
 * sink buffer for the call.
 * fp8_ubench_lds: waves_per_cu waves per CU each read 16 bytes per lane
 * (ds_read_b128, conflict-free) `iters` times; bytes = CUs x waves x 64 x 16
 * x iters.
 * fp8_ubench_lds_pattern: the same with the address pattern of a GEMM
 * fragment read (lane l reads row l % 16 of a 16-row block at chunk position
 * l / 16; each iteration moves to the next block): 0 linear (= fp8_ubench_lds),
 * 1 dense operand (128-byte swizzled rows, 16 bytes at chunk 2 (l/16)),
 * 2 compressed operand (64-byte swizzled rows), 3 dense B operand of the 2:4
 * kernels at its chunk positions (l/16 + 4) and swizzle, 4 metadata (16-byte
 * rows, 4 bytes per lane: ds_read_b32), 5 compressed operand without swizzle,
 * 6 metadata of two 16-row blocks in one instruction (8 bytes per lane,
 * ds_read2st64_b32), 7 the read of 3 on the dense kernels' swizzle.  Bank
 * conflicts of a pattern appear as a longer time (and in the LDS conflict
 * counters).  Patterns outside 0..7 are rejected with FP8_ERR_ARG. */
fp8_status fp8_ubench_mfma(int kind, int waves_per_cu, int chains, int iters, void *stream, double *ms);
fp8_status fp8_ubench_lds(int waves_per_cu, int iters, void *stream, double *ms);
fp8_status fp8_ubench_lds_pattern(int pattern, int waves_per_cu, int iters, void *stream, double *ms);
/* Any 128-bit read (write = 0) or write (write = 1) pattern: lane l of every
 * wave accesses 16 bytes at lane_offsets[l] (64 host ints, 16-byte aligned,
 * below 32768) plus a per-iteration shift of a multiple of 2 KiB; times as
 * above.  A lane pattern whose accesses collide in a bank takes longer, so
 * lane groupings and bank mappings can be probed.  FP8_ERR_ARG for offsets
 * outside that range. */
fp8_status fp8_ubench_lds_offsets(const int *lane_offsets, int write, int waves_per_cu, int iters, void *stream,
                                  double *ms);
/* The engine clock under matrix-core load (the clock the measured MFMA rates
 * run at, against the 2.4 GHz the peak figures assume): 8 waves per CU run the
 * 16x16x128 FP8 MFMA loop for `iters` rounds of 8 instructions while one wave
 * reads the shader clock counter and the constant-rate wall clock before and
 * after; *ghz = clock ticks / wall seconds.  Blocking; allocates two small
 * buffers for the call.  FP8_ERR_UNSUPPORTED if the device reports no wall
 * clock rate. */
fp8_status fp8_ubench_clock(int iters, void *stream, double *ghz);

/* ------------------------------------------------------------------------ */
/* Validator support: FP64 error norms on the device.                        */
/* ------------------------------------------------------------------------ */
/* Given the device result c (FP32 or BF16, M x N, ldc) and FP64 references
 * cref, sabs (M x N, packed), accumulates over all elements:
 *   out[0] = max |c - cref|, out[1] = max |c - cref| / bound,
 *   out[2] = sum (c - cref)^2, out[3] = sum cref^2, out[4] = count over bound
 * where bound = 4 K 2^-24 sabs (FP32) or (1 + 2^-8) 4 K 2^-24 sabs + 2^-8 |cref|
 * (BF16).  out: 5 device doubles.  FP64 is used here only, never in a GEMM. */
fp8_status fp8_validate(const void *c, fp8_out c_type, int64_t ldc, const double *cref,
                        const double *sabs, int64_t M, int64_t N, int64_t K, double *out,
                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FP8GEMM_H */
