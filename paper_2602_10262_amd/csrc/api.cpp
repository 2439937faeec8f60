// C ABI of libfp8gemm.so: argument checks, plan choice and dispatch for
// quantize, prune/compress, dense and 2:4 GEMM, validation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "api_util.hpp"

namespace fp8k {

static thread_local std::string g_err;

fp8_status set_error(fp8_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

fp8_status hip_error(hipError_t e, const char *what)
{
    return set_error(FP8_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
static bool fmt_ok(int f) { return f == FP8_E4M3 || f == FP8_E5M2; }
static inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static const int64_t kMaxDim = (int64_t)1 << 30;
// Kernels address a tile's rows with 32-bit buffer offsets: 256 rows of the
// largest leading dimension must stay below 2^31 bytes.
static const int64_t kMaxLd = (int64_t)1 << 22;

// Common checks of the dense description (the sparse side's operand is
// checked by the caller instead).
static fp8_status check_common(const fp8_gemm_args *a, bool need_a, bool need_b)
{
    if (!a) return set_error(FP8_ERR_ARG, "null args");
    if (a->M < 1 || a->N < 1 || a->K < 1 || a->M > kMaxDim || a->N > kMaxDim || a->K > kMaxDim)
        return set_error(FP8_ERR_SHAPE, "M, N, K must be in [1, 2^30]");
    if ((int64_t)a->M * a->N > ((int64_t)1 << 40)) return set_error(FP8_ERR_SHAPE, "M*N too large");
    if (!fmt_ok(a->a_fmt) || !fmt_ok(a->b_fmt)) return set_error(FP8_ERR_ARG, "unknown FP8 format");
    if (a->c_type != FP8_OUT_F32 && a->c_type != FP8_OUT_BF16 && a->c_type != FP8_OUT_F16)
        return set_error(FP8_ERR_ARG, "unknown output type");
    if ((a->a_kind != FP8_SCALE_TENSOR && a->a_kind != FP8_SCALE_ROW) ||
        (a->b_kind != FP8_SCALE_TENSOR && a->b_kind != FP8_SCALE_ROW))
        return set_error(FP8_ERR_ARG, "unknown scale kind");
    if (!a->a_descale || !a->b_descale || !a->c) return set_error(FP8_ERR_ARG, "null descale or output pointer");
    if (a->ldc < a->N) return set_error(FP8_ERR_ARG, "ldc < N");
    if (a->K > kMaxLd || (need_a && a->lda > kMaxLd) || (need_b && a->ldb > kMaxLd))
        return set_error(FP8_ERR_SHAPE, "K and leading dimensions must be <= 4194304");
    if (need_a) {
        if (!a->a) return set_error(FP8_ERR_ARG, "null A");
        if (a->lda < a->K) return set_error(FP8_ERR_ARG, "lda < K");
        if (!aligned16(a->a) || a->lda % 16) return set_error(FP8_ERR_ALIGN, "A pointer and lda must be 16-byte aligned");
    }
    if (need_b) {
        if (!a->b) return set_error(FP8_ERR_ARG, "null B");
        if (a->ldb < a->K) return set_error(FP8_ERR_ARG, "ldb < K");
        if (!aligned16(a->b) || a->ldb % 16) return set_error(FP8_ERR_ALIGN, "B pointer and ldb must be 16-byte aligned");
    }
    return FP8_OK;
}

fp8_status prepare_dense(const fp8_gemm_args *a, Prepared &out)
{
    fp8_status st = check_common(a, true, true);
    if (st != FP8_OK) return st;
    GemmParams &p = out.p;
    std::memset(&p, 0, sizeof(p));
    p.a = a->a; p.lda = a->lda;
    p.b = a->b; p.ldb = a->ldb;
    p.si = a->a_descale; p.si_per = a->a_kind == FP8_SCALE_ROW;
    p.sj = a->b_descale; p.sj_per = a->b_kind == FP8_SCALE_ROW;
    p.c = a->c; p.ldc = a->ldc; p.out_bf16 = a->c_type == FP8_OUT_BF16; p.out_f16 = a->c_type == FP8_OUT_F16; p.trans_out = 0;
    p.M = (int)a->M; p.N = (int)a->N; p.K = (int)a->K;
    p.splits = 1; p.kchunk = ((p.K + kBKHost - 1) / kBKHost) * kBKHost;
    out.fa = a->a_fmt; out.fb = a->b_fmt; out.sparse = false;
    out.key = GemmKey{a->M, a->N, a->K, out.fa, out.fb, (int)a->c_type, p.si_per, p.sj_per, 0};
    return FP8_OK;
}

fp8_status prepare_sparse(const fp8_sparse24_gemm_args *s, Prepared &out)
{
    if (!s) return set_error(FP8_ERR_ARG, "null args");
    const fp8_gemm_args *a = &s->g;
    const bool side_a = s->side == FP8_SPARSE_A;
    if (s->side != FP8_SPARSE_A && s->side != FP8_SPARSE_B) return set_error(FP8_ERR_ARG, "unknown sparse side");
    fp8_status st = check_common(a, !side_a, side_a);
    if (st != FP8_OK) return st;
    if (a->K % 8) return set_error(FP8_ERR_SHAPE, "2:4 GEMM needs K % 8 == 0");
    if (!s->values || !s->meta) return set_error(FP8_ERR_ARG, "null compressed operand");
    if (!aligned16(s->values) || !aligned16(s->meta))
        return set_error(FP8_ERR_ALIGN, "compressed values and metadata must be 16-byte aligned");
    GemmParams &p = out.p;
    std::memset(&p, 0, sizeof(p));
    p.a = s->values; p.lda = a->K / 2;
    p.meta = s->meta; p.ldm = a->K / 8;
    p.c = a->c; p.ldc = a->ldc; p.out_bf16 = a->c_type == FP8_OUT_BF16; p.out_f16 = a->c_type == FP8_OUT_F16;
    p.K = (int)a->K;
    p.splits = 1; p.kchunk = ((p.K + kBKHost - 1) / kBKHost) * kBKHost;
    if (side_a) {
        p.b = a->b; p.ldb = a->ldb;
        p.si = a->a_descale; p.si_per = a->a_kind == FP8_SCALE_ROW;
        p.sj = a->b_descale; p.sj_per = a->b_kind == FP8_SCALE_ROW;
        p.M = (int)a->M; p.N = (int)a->N; p.trans_out = 0;
        out.fa = a->a_fmt; out.fb = a->b_fmt;
    } else {
        // C^T = W A^T: the compressed weight rows take the MFMA A slot.
        p.b = a->a; p.ldb = a->lda;
        p.si = a->b_descale; p.si_per = a->b_kind == FP8_SCALE_ROW;
        p.sj = a->a_descale; p.sj_per = a->a_kind == FP8_SCALE_ROW;
        p.M = (int)a->N; p.N = (int)a->M; p.trans_out = 1;
        out.fa = a->b_fmt; out.fb = a->a_fmt;
    }
    out.sparse = true;
    out.key = GemmKey{p.M, p.N, a->K, out.fa, out.fb, (int)a->c_type, p.si_per, p.sj_per, side_a ? 1 : 2};
    return FP8_OK;
}

void apply_split(GemmParams &p, int split_k)
{
    const int steps = (p.K + kBKHost - 1) / kBKHost;
    int s = std::max(1, std::min(split_k, steps));
    const int per = (steps + s - 1) / s;
    s = (steps + per - 1) / per;   // no empty split
    p.splits = s;
    p.kchunk = per * kBKHost;
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Split count that brings a grid of nb tiles to about two workgroups per CU
// while keeping at least four K steps per split.
static int default_splits(int64_t nb, int64_t K)
{
    const int64_t steps = cdiv(K, kBKHost);
    int64_t want = 1;
    if (nb < 256) want = std::min<int64_t>(cdiv(512, nb), std::max<int64_t>(1, steps / 4));
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, 64));
}

fp8_plan heuristic_plan(const GemmKey &k)
{
    fp8_plan p;
    const int64_t M = k.mk, N = k.nk;
    if (k.kk < kExactBelowK) {
        // exact-sum tiles.  K in whole 16-byte chunks (128 codes with a 2:4
        // operand): the 256 x 256 DMA-ring tile from about half a chip of
        // such tiles, without split-K (measured dense 3072^3: 75 us vs 86 for
        // 128 x 128 and 123 split four ways; 8192^2 x 2048: 226 vs 321; 2:4
        // 314 vs 425 on the register tile).  Then 128 x 128 from a full chip
        // of those: the DMA ring for dense operands (2048^3: 24 us vs 30),
        // the register tile for a 2:4 one (31 us vs 37: the expansion after
        // the fragment reads costs more than the ring saves).  Otherwise the
        // 64 x 64 register tile (split-K below adds workgroups; 1024^3: 10
        // us vs 14).
        const bool dma = (k.kk % (k.sparse ? 128 : 16)) == 0;
        if (dma && cdiv(M, 256) * cdiv(N, 256) >= 128) {
            p.tile = 30;
            p.split_k = 1;
            return p;
        }
        if (cdiv(M, 128) * cdiv(N, 128) >= 256) p.tile = (dma && !k.sparse) ? 28 : 27;
        else p.tile = 26;
        const TileDesc &t = tile_desc(p.tile);
        p.split_k = default_splits(cdiv(M, t.bm) * cdiv(N, t.bn), k.kk);
        return p;
    }
    if (N <= 16) p.tile = 8;
    else if (N <= 32) p.tile = 9;
    // single-wave 16 x 32 tiles on a 12-stage DMA ring: enough workgroups
    // without split-K once N is large
    else if (!k.sparse && M <= 16 && N >= 4096 && (k.kk % 16) == 0) p.tile = 24;
    else if (M <= 16) p.tile = 4;
    else if (M <= 32) p.tile = 5;
    else if (M <= 64) p.tile = 7;
    else if (M <= 128 || N <= 128) p.tile = 0;
    // up to 1024 x 1024 outputs: 128 x 16 tiles give 8x the workgroups of
    // 128 x 128 (measured 10.3 vs 16.2 us at 1024^3), dense and 2:4 alike
    else if (M * N <= (int64_t)1024 * 1024) p.tile = 8;
    // 256 x 256 with LDS DMA: 128 x 64 wave tiles read 25% less LDS per
    // MFMA than 64 x 64 ones and no registers stage the loads; it wins once
    // there are enough tiles to fill the chip
    else if (M >= 4096 && N >= 4096 && (k.kk % 128) == 0) p.tile = 19;
    else if (M * N >= (int64_t)4096 * 4096) p.tile = N >= M ? 13 : 12;
    else p.tile = 0;
    const TileDesc &t = tile_desc(p.tile);
    p.split_k = default_splits(cdiv(M, t.bm) * cdiv(N, t.bn), k.kk);
    return p;
}

fp8_status resolve_plan(const Prepared &pr, const fp8_plan *plan, fp8_plan &res)
{
    if (!tune_cache_lookup(pr.key, res)) res = heuristic_plan(pr.key);
    if (plan) {
        if (plan->tile >= num_tiles()) return set_error(FP8_ERR_ARG, "plan.tile out of range");
        if (plan->tile >= 0) {
            if (pr.sparse && !tile_desc(plan->tile).sparse_ok)
                return set_error(FP8_ERR_ARG, "plan.tile has no 2:4 kernel");
            if (!pr.sparse && !tile_desc(plan->tile).dense_ok)
                return set_error(FP8_ERR_ARG, "plan.tile has no dense kernel");
            res.tile = plan->tile;
            const TileDesc &t = tile_desc(res.tile);
            res.split_k = default_splits(cdiv(pr.key.mk, t.bm) * cdiv(pr.key.nk, t.bn), pr.key.kk);
        }
        if (plan->split_k > 0) res.split_k = plan->split_k;
    }
    if (res.split_k < 1) res.split_k = 1;
    GemmParams p = pr.p;
    apply_split(p, res.split_k);
    res.split_k = p.splits;
    return FP8_OK;
}

size_t workspace_bytes(const Prepared &pr, const fp8_plan &res)
{
    GemmParams p = pr.p;
    apply_split(p, res.split_k);
    if (p.splits <= 1) return 0;
    return (size_t)p.splits * (size_t)p.M * (size_t)p.N * sizeof(float);
}

fp8_status run_prepared(Prepared pr, const fp8_plan &res, void *ws, size_t ws_bytes, hipStream_t st)
{
    apply_split(pr.p, res.split_k);
    const size_t need = workspace_bytes(pr, res);
    if (need > 0) {
        if (!ws || ws_bytes < need) return set_error(FP8_ERR_ARG, "workspace too small: need " + std::to_string(need));
        pr.p.ws = static_cast<float *>(ws);
    }
    hipError_t e = launch_gemm(res.tile, pr.fa, pr.fb, pr.sparse, pr.p, st);
    if (e != hipSuccess) return hip_error(e, "gemm launch");
    if (pr.p.splits > 1) {
        e = launch_splitk_reduce(pr.p, st);
        if (e != hipSuccess) return hip_error(e, "split-K reduce launch");
    }
    return FP8_OK;
}

}  // namespace fp8k

using namespace fp8k;

extern "C" {

const char *fp8_last_error(void) { return g_err.c_str(); }
int fp8_version(void) { return 1; }

fp8_status fp8_quantize_workspace_size(int64_t rows, int64_t cols, fp8_scale_kind kind, size_t *bytes)
{
    if (!bytes) return set_error(FP8_ERR_ARG, "null bytes");
    if (rows < 1 || cols < 1) return set_error(FP8_ERR_SHAPE, "rows, cols must be >= 1");
    *bytes = kind == FP8_SCALE_TENSOR ? 4 : 0;
    return FP8_OK;
}

fp8_status fp8_quantize(const float *x, int64_t rows, int64_t cols, int64_t ldx, fp8_fmt fmt, fp8_scale_kind kind,
                        uint8_t *q, int64_t ldq, float *scale, float *descale, void *ws, size_t ws_bytes,
                        void *stream)
{
    if (!x || !q || !scale || !descale) return set_error(FP8_ERR_ARG, "null pointer");
    if (rows < 1 || cols < 1 || rows > kMaxDim || cols > kMaxDim) return set_error(FP8_ERR_SHAPE, "rows, cols out of range");
    if (!fmt_ok(fmt)) return set_error(FP8_ERR_ARG, "unknown FP8 format");
    if (kind != FP8_SCALE_TENSOR && kind != FP8_SCALE_ROW) return set_error(FP8_ERR_ARG, "unknown scale kind");
    if (ldx < cols || ldq < cols) return set_error(FP8_ERR_ARG, "leading dimension < cols");
    if (!aligned16(x) || ldx % 4) return set_error(FP8_ERR_ALIGN, "x must be 16-byte aligned with ldx % 4 == 0");
    if (!aligned16(q) || ldq % 16) return set_error(FP8_ERR_ALIGN, "q must be 16-byte aligned with ldq % 16 == 0");
    if (kind == FP8_SCALE_TENSOR && (!ws || ws_bytes < 4)) return set_error(FP8_ERR_ARG, "workspace too small: need 4");
    hipError_t e = launch_quantize(x, rows, cols, ldx, fmt, kind == FP8_SCALE_ROW, q, ldq, scale, descale, ws,
                                   as_stream(stream));
    if (e != hipSuccess) return hip_error(e, "quantize launch");
    return FP8_OK;
}

fp8_status fp8_tile_info(int tile, int *block_m, int *block_n, int *waves, int *sparse, int *dense, int *exact)
{
    if (tile < 0 || tile >= num_tiles()) return set_error(FP8_ERR_ARG, "tile out of range");
    const TileDesc &t = tile_desc(tile);
    if (block_m) *block_m = t.bm;
    if (block_n) *block_n = t.bn;
    if (waves) *waves = t.waves;
    if (sparse) *sparse = t.sparse_ok;
    if (dense) *dense = t.dense_ok;
    if (exact) *exact = t.exact;
    return FP8_OK;
}

int fp8_num_tiles(void) { return num_tiles(); }

fp8_status fp8_gemm_plan_resolve(const fp8_gemm_args *args, const fp8_plan *plan, fp8_plan *resolved)
{
    if (!resolved) return set_error(FP8_ERR_ARG, "null resolved");
    Prepared pr;
    fp8_status st = prepare_dense(args, pr);
    if (st != FP8_OK) return st;
    return resolve_plan(pr, plan, *resolved);
}

fp8_status fp8_gemm_workspace_size(const fp8_gemm_args *args, const fp8_plan *plan, size_t *bytes)
{
    if (!bytes) return set_error(FP8_ERR_ARG, "null bytes");
    Prepared pr;
    fp8_status st = prepare_dense(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_plan(pr, plan, res);
    if (st != FP8_OK) return st;
    *bytes = workspace_bytes(pr, res);
    return FP8_OK;
}

fp8_status fp8_gemm(const fp8_gemm_args *args, const fp8_plan *plan, void *ws, size_t ws_bytes, void *stream)
{
    Prepared pr;
    fp8_status st = prepare_dense(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_plan(pr, plan, res);
    if (st != FP8_OK) return st;
    return run_prepared(pr, res, ws, ws_bytes, as_stream(stream));
}

fp8_status fp8_sparse24_prune_compress(const uint8_t *x, fp8_fmt fmt, int64_t rows, int64_t K, int64_t ldx,
                                       uint8_t *values, uint8_t *meta, uint8_t *mask, void *stream)
{
    if (!x || !values || !meta) return set_error(FP8_ERR_ARG, "null pointer");
    if (!fmt_ok(fmt)) return set_error(FP8_ERR_ARG, "unknown FP8 format");
    if (rows < 1 || K < 1 || rows > kMaxDim || K > kMaxDim) return set_error(FP8_ERR_SHAPE, "rows, K out of range");
    if (K % 8) return set_error(FP8_ERR_SHAPE, "K % 8 != 0");
    if (ldx < K) return set_error(FP8_ERR_ARG, "ldx < K");
    if (!aligned16(x) || ldx % 16 || !aligned16(values) || !aligned16(meta) || (mask && !aligned16(mask)))
        return set_error(FP8_ERR_ALIGN, "pointers and ldx must be 16-byte aligned");
    hipError_t e = launch_prune24(x, rows, K, ldx, values, meta, mask, as_stream(stream));
    if (e != hipSuccess) return hip_error(e, "prune launch");
    return FP8_OK;
}

fp8_status fp8_quantize_prune24(const float *x, int64_t rows, int64_t K, int64_t ldx, fp8_fmt fmt,
                                fp8_scale_kind kind, uint8_t *values, uint8_t *meta, uint8_t *mask, float *scale,
                                float *descale, void *ws, size_t ws_bytes, void *stream)
{
    if (!x || !values || !meta || !scale || !descale) return set_error(FP8_ERR_ARG, "null pointer");
    if (rows < 1 || K < 1 || rows > kMaxDim || K > kMaxDim) return set_error(FP8_ERR_SHAPE, "rows, K out of range");
    if (K % 8) return set_error(FP8_ERR_SHAPE, "K % 8 != 0");
    if (!fmt_ok(fmt)) return set_error(FP8_ERR_ARG, "unknown FP8 format");
    if (kind != FP8_SCALE_TENSOR && kind != FP8_SCALE_ROW) return set_error(FP8_ERR_ARG, "unknown scale kind");
    if (ldx < K) return set_error(FP8_ERR_ARG, "ldx < K");
    if (!aligned16(x) || ldx % 4) return set_error(FP8_ERR_ALIGN, "x must be 16-byte aligned with ldx % 4 == 0");
    if (!aligned16(values) || !aligned16(meta) || (mask && !aligned16(mask)))
        return set_error(FP8_ERR_ALIGN, "values, meta and mask must be 16-byte aligned");
    if (kind == FP8_SCALE_TENSOR && (!ws || ws_bytes < 4)) return set_error(FP8_ERR_ARG, "workspace too small: need 4");
    hipError_t e = launch_quantize_prune24(x, rows, K, ldx, fmt, kind == FP8_SCALE_ROW, values, meta, mask, scale,
                                           descale, ws, as_stream(stream));
    if (e != hipSuccess) return hip_error(e, "quantize+prune launch");
    return FP8_OK;
}

fp8_status fp8_sparse24_decompress(const uint8_t *values, const uint8_t *meta, int64_t rows, int64_t K, uint8_t *out,
                                   int64_t ldo, void *stream)
{
    if (!values || !meta || !out) return set_error(FP8_ERR_ARG, "null pointer");
    if (rows < 1 || K < 1 || rows > kMaxDim || K > kMaxDim) return set_error(FP8_ERR_SHAPE, "rows, K out of range");
    if (K % 8) return set_error(FP8_ERR_SHAPE, "K % 8 != 0");
    if (ldo < K) return set_error(FP8_ERR_ARG, "ldo < K");
    hipError_t e = launch_decompress24(values, meta, rows, K, out, ldo, as_stream(stream));
    if (e != hipSuccess) return hip_error(e, "decompress launch");
    return FP8_OK;
}

fp8_status fp8_sparse24_gemm_workspace_size(const fp8_sparse24_gemm_args *args, const fp8_plan *plan, size_t *bytes)
{
    if (!bytes) return set_error(FP8_ERR_ARG, "null bytes");
    Prepared pr;
    fp8_status st = prepare_sparse(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_plan(pr, plan, res);
    if (st != FP8_OK) return st;
    *bytes = workspace_bytes(pr, res);
    return FP8_OK;
}

fp8_status fp8_sparse24_gemm(const fp8_sparse24_gemm_args *args, const fp8_plan *plan, void *ws, size_t ws_bytes,
                             void *stream)
{
    Prepared pr;
    fp8_status st = prepare_sparse(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_plan(pr, plan, res);
    if (st != FP8_OK) return st;
    return run_prepared(pr, res, ws, ws_bytes, as_stream(stream));
}

// ---- both operands 2:4-compressed ----------------------------------------

// Kernel view: the compressed activations take the SMFMAC slot (i = rows of
// A) unless A has fewer than 64 rows and the weight at least 64, in which case
// the weight rows do and the output is stored transposed, as in the
// weight-side 2:4 GEMM.
static fp8_status prepare_both(const fp8_sparse24_both_gemm_args *s, Prepared &out)
{
    if (!s) return set_error(FP8_ERR_ARG, "null args");
    const fp8_gemm_args *a = &s->g;
    fp8_status st = check_common(a, false, false);
    if (st != FP8_OK) return st;
    if (a->K % 8) return set_error(FP8_ERR_SHAPE, "2:4 GEMM needs K % 8 == 0");
    if (!s->a_values || !s->a_meta || !s->b_values || !s->b_meta)
        return set_error(FP8_ERR_ARG, "null compressed operand");
    if (!aligned16(s->a_values) || !aligned16(s->a_meta) || !aligned16(s->b_values) || !aligned16(s->b_meta))
        return set_error(FP8_ERR_ALIGN, "compressed values and metadata must be 16-byte aligned");
    const bool swap = a->M < 64 && a->N >= 64;
    GemmParams &p = out.p;
    std::memset(&p, 0, sizeof(p));
    p.lda = p.ldb = a->K / 2;
    p.ldm = p.ldmb = a->K / 8;
    p.c = a->c; p.ldc = a->ldc; p.out_bf16 = a->c_type == FP8_OUT_BF16; p.out_f16 = a->c_type == FP8_OUT_F16;
    p.K = (int)a->K;
    p.splits = 1; p.kchunk = ((p.K + kBKHost - 1) / kBKHost) * kBKHost;
    if (!swap) {
        p.a = s->a_values; p.meta = s->a_meta;
        p.b = s->b_values; p.meta_b = s->b_meta;
        p.si = a->a_descale; p.si_per = a->a_kind == FP8_SCALE_ROW;
        p.sj = a->b_descale; p.sj_per = a->b_kind == FP8_SCALE_ROW;
        p.M = (int)a->M; p.N = (int)a->N; p.trans_out = 0;
        out.fa = a->a_fmt; out.fb = a->b_fmt;
    } else {
        p.a = s->b_values; p.meta = s->b_meta;
        p.b = s->a_values; p.meta_b = s->a_meta;
        p.si = a->b_descale; p.si_per = a->b_kind == FP8_SCALE_ROW;
        p.sj = a->a_descale; p.sj_per = a->a_kind == FP8_SCALE_ROW;
        p.M = (int)a->N; p.N = (int)a->M; p.trans_out = 1;
        out.fa = a->b_fmt; out.fb = a->a_fmt;
    }
    out.sparse = true;
    out.key = GemmKey{p.M, p.N, a->K, out.fa, out.fb, (int)a->c_type, p.si_per, p.sj_per, 3};
    return FP8_OK;
}

static fp8_status resolve_both(const Prepared &pr, const fp8_plan *plan, fp8_plan &res)
{
    const int64_t M = pr.p.M, N = pr.p.N, K = pr.p.K;
    if (K < kExactBelowK) res.tile = cdiv(M, 128) * cdiv(N, 128) >= 256 ? 27 : 26;
    else if (M >= 4096 && N >= 4096) res.tile = 12;
    else if (M <= 64 || N <= 64) res.tile = 3;
    else res.tile = 0;
    if (plan && plan->tile >= 0) {
        if (!both_tile_supported(plan->tile)) return set_error(FP8_ERR_ARG, "plan.tile has no both-sides 2:4 kernel");
        res.tile = plan->tile;
    }
    const TileDesc &t = tile_desc(res.tile);
    res.split_k = default_splits(cdiv(M, t.bm) * cdiv(N, t.bn), K);
    if (plan && plan->split_k > 0) res.split_k = plan->split_k;
    GemmParams p = pr.p;
    apply_split(p, res.split_k);
    res.split_k = p.splits;
    return FP8_OK;
}

fp8_status fp8_sparse24_both_gemm_workspace_size(const fp8_sparse24_both_gemm_args *args, const fp8_plan *plan,
                                                 size_t *bytes)
{
    if (!bytes) return set_error(FP8_ERR_ARG, "null bytes");
    Prepared pr;
    fp8_status st = prepare_both(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_both(pr, plan, res);
    if (st != FP8_OK) return st;
    *bytes = workspace_bytes(pr, res);
    return FP8_OK;
}

fp8_status fp8_sparse24_both_gemm_plan_resolve(const fp8_sparse24_both_gemm_args *args, const fp8_plan *plan,
                                               fp8_plan *resolved)
{
    if (!resolved) return set_error(FP8_ERR_ARG, "null resolved");
    Prepared pr;
    fp8_status st = prepare_both(args, pr);
    if (st != FP8_OK) return st;
    return resolve_both(pr, plan, *resolved);
}

fp8_status fp8_sparse24_both_gemm(const fp8_sparse24_both_gemm_args *args, const fp8_plan *plan, void *ws,
                                  size_t ws_bytes, void *stream)
{
    Prepared pr;
    fp8_status st = prepare_both(args, pr);
    if (st != FP8_OK) return st;
    fp8_plan res;
    st = resolve_both(pr, plan, res);
    if (st != FP8_OK) return st;
    apply_split(pr.p, res.split_k);
    const size_t need = workspace_bytes(pr, res);
    if (need > 0) {
        if (!ws || ws_bytes < need) return set_error(FP8_ERR_ARG, "workspace too small: need " + std::to_string(need));
        pr.p.ws = static_cast<float *>(ws);
    }
    const hipStream_t hs = as_stream(stream);
    hipError_t e = launch_gemm_both(res.tile, pr.fa, pr.fb, pr.p, hs);
    if (e != hipSuccess) return hip_error(e, "both-sides 2:4 gemm launch");
    if (pr.p.splits > 1) {
        e = launch_splitk_reduce(pr.p, hs);
        if (e != hipSuccess) return hip_error(e, "split-K reduce launch");
    }
    return FP8_OK;
}

fp8_status fp8_validate(const void *c, fp8_out c_type, int64_t ldc, const double *cref, const double *sabs, int64_t M,
                        int64_t N, int64_t K, double *out, void *stream)
{
    if (!c || !cref || !sabs || !out) return set_error(FP8_ERR_ARG, "null pointer");
    if (M < 1 || N < 1 || K < 1) return set_error(FP8_ERR_SHAPE, "M, N, K must be >= 1");
    if (ldc < N) return set_error(FP8_ERR_ARG, "ldc < N");
    hipError_t e = launch_validate(c, c_type == FP8_OUT_BF16, ldc, cref, sabs, M, N, K, out, as_stream(stream));
    if (e != hipSuccess) return hip_error(e, "validate launch");
    return FP8_OK;
}

}  // extern "C"
