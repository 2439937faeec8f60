/*
 * Plain, slow CPU oracle for the FP8 GEMM hot path.  TEST INFRASTRUCTURE ONLY:
 * it is called by the test suite, by the smoke check and by the CPU-baseline
 * leg of the benchmark, never by the library.  It shares no code with the GPU
 * path and includes nothing from it.
 *
 * What it computes (paper: arXiv 2602.10262, "Execution-Centric
 * Characterization of FP8 Matrix Cores, Asynchronous Execution, and Structured
 * Sparsity on AMD MI300A"):
 *   - FP8 operands in the two OCP 8-bit formats the paper names (E4M3 and
 *     E5M2), multiplied with FP32 accumulation on the GPU (Sec. 2, "FP8 Matrix
 *     Cores"); here every code is decoded exactly to FP64 and every product
 *     and sum is done in FP64.
 *   - 2:4 structured sparsity along the reduction dimension: two of every
 *     four consecutive elements are zero (Sec. 2, "Structured Sparsity";
 *     Sec. 7 opening paragraph).  Which two survive is the rule stated in the
 *     header of orc_prune24 below.
 *   - Per-tensor and per-row scales derived from amax (the "wavefront-level
 *     reductions for amax and scales" of the method statement), so that the
 *     FP8 range is filled by scaling.
 *
 * Every function is the plain definition written out: no blocking, no fused
 * loops, no reordering beyond what the definition allows.  Formats: 0 = E4M3,
 * 1 = E5M2 (OCP encodings, not the FNUZ ones of gfx942).
 *
 * Parity status: every function here is pinned by tests against values fixed
 * by the OCP format definition, by an independent library decoder, by exact
 * rational arithmetic on small inputs, by exhaustive enumeration and by
 * closed forms.  No function is "parity unpinned".
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_E4M3 0
#define ORC_E5M2 1

/* ------------------------------------------------------------------------- */
/* Decode: OCP 8-bit floating point, exactly to FP64.                          */
/* ------------------------------------------------------------------------- */

/* E4M3: sign, 4 exponent bits (bias 7), 3 mantissa bits; subnormals at
 * exponent field 0; S.1111.111 is NaN; there is no infinity.
 * E5M2: sign, 5 exponent bits (bias 15), 2 mantissa bits; IEEE-style
 * infinities (exponent all ones, mantissa 0) and NaNs. */
double orc_decode(int fmt, uint8_t code)
{
    int s = code >> 7;
    double sign = s ? -1.0 : 1.0;
    if (fmt == ORC_E4M3) {
        int e = (code >> 3) & 0xF, m = code & 0x7;
        if (e == 15 && m == 7) return NAN;
        if (e == 0) return sign * ldexp((double)m, -9);           /* m/8 * 2^(1-7) */
        return sign * ldexp(1.0 + m / 8.0, e - 7);
    } else {
        int e = (code >> 2) & 0x1F, m = code & 0x3;
        if (e == 31) return m == 0 ? sign * INFINITY : NAN;
        if (e == 0) return sign * ldexp((double)m, -16);          /* m/4 * 2^(1-15) */
        return sign * ldexp(1.0 + m / 4.0, e - 15);
    }
}

static uint8_t max_finite_code(int fmt) { return fmt == ORC_E4M3 ? 0x7E : 0x7B; }

double orc_max_finite(int fmt) { return orc_decode(fmt, max_finite_code(fmt)); }

/* ------------------------------------------------------------------------- */
/* Encode FP32 -> FP8: round to nearest, ties to even, saturating.             */
/* ------------------------------------------------------------------------- */

/* The definition: the exact real value of x (an FP32 value is exact in FP64)
 * goes to the finite FP8 value nearest to it; an exact tie goes to the code
 * whose mantissa LSB is 0 (the even code); anything beyond the largest finite
 * magnitude, infinities included, goes to that largest magnitude (saturation).
 * The sign is kept, so a negative value that rounds to zero is -0 (0x80).
 * NaN goes to 0x7F with the sign of the input (a NaN code in both formats).
 * Implemented as a binary search over the ascending table of finite
 * non-negative values. */
uint8_t orc_encode(int fmt, float x)
{
    uint32_t bits;
    memcpy(&bits, &x, 4);
    uint8_t sign = (uint8_t)((bits >> 31) << 7);
    if (isnan(x)) return (uint8_t)(0x7F | sign);
    double ax = fabs((double)x);
    int top = max_finite_code(fmt);
    if (ax >= orc_decode(fmt, (uint8_t)top)) return (uint8_t)(top | sign);
    /* Largest code lo with decode(lo) <= ax; codes 0..top are ascending. */
    int lo = 0, hi = top;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (orc_decode(fmt, (uint8_t)mid) <= ax) lo = mid; else hi = mid;
    }
    /* The midpoint of two adjacent FP8 values is exact in FP64. */
    double mid = 0.5 * (orc_decode(fmt, (uint8_t)lo) + orc_decode(fmt, (uint8_t)hi));
    int pick;
    if (ax < mid) pick = lo;
    else if (ax > mid) pick = hi;
    else pick = (lo % 2 == 0) ? lo : hi;
    return (uint8_t)(pick | sign);
}

/* A second encoder written independently from the first (integer rounding of
 * the FP32 significand), used only to cross-check orc_encode exhaustively over
 * all 2^32 FP32 bit patterns. */
uint8_t orc_encode_bitwise(int fmt, float x)
{
    const int M = fmt == ORC_E4M3 ? 3 : 2;
    const int B = fmt == ORC_E4M3 ? 7 : 15;
    const uint32_t top = max_finite_code(fmt);
    uint32_t bits;
    memcpy(&bits, &x, 4);
    uint32_t sign = (bits >> 31) << 7;
    uint32_t a = bits & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (uint8_t)(0x7F | sign);
    if (a == 0x7F800000u) return (uint8_t)(top | sign);
    int e32 = (int)(a >> 23) - 127;
    uint32_t sig = a & 0x7FFFFFu;
    if ((a >> 23) == 0) e32 = -126; else sig |= 0x800000u;
    uint32_t code, rem, half;
    int sh;
    if (e32 >= 1 - B) {
        /* normal FP8 range: keep M fraction bits; carry into the exponent
         * field happens by plain integer addition */
        sh = 23 - M;
        code = ((uint32_t)(e32 + B) << M) + ((sig & 0x7FFFFFu) >> sh);
    } else {
        /* subnormal FP8 range: units of 2^(1-B-M) */
        sh = 23 + 1 - B - M - e32;
        if (sh > 30) return (uint8_t)sign;
        code = sig >> sh;
    }
    rem = sig & ((1u << sh) - 1u);
    half = 1u << (sh - 1);
    if (rem > half || (rem == half && (code & 1u))) code += 1;
    if (code > top) code = top;
    return (uint8_t)(code | sign);
}

typedef struct {
    int fmt;
    uint64_t lo, hi;
    uint64_t bad;
    uint32_t first_bad;
} sweep_job;

static void *sweep_worker(void *p)
{
    sweep_job *j = (sweep_job *)p;
    j->bad = 0;
    j->first_bad = 0;
    for (uint64_t u = j->lo; u < j->hi; ++u) {
        uint32_t b = (uint32_t)u;
        float x;
        memcpy(&x, &b, 4);
        if (orc_encode(j->fmt, x) != orc_encode_bitwise(j->fmt, x)) {
            if (j->bad == 0) j->first_bad = b;
            j->bad++;
        }
    }
    return NULL;
}

/* Compare the two encoders on every FP32 bit pattern in [lo, hi).  Returns the
 * number of disagreements; *first_bad receives the first one. */
uint64_t orc_encode_sweep(int fmt, uint64_t lo, uint64_t hi, int nthreads, uint32_t *first_bad)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    sweep_job jobs[256];
    uint64_t span = hi - lo, step = (span + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fmt = fmt;
        jobs[t].lo = lo + step * t < hi ? lo + step * t : hi;
        jobs[t].hi = lo + step * (t + 1) < hi ? lo + step * (t + 1) : hi;
        pthread_create(&th[t], NULL, sweep_worker, &jobs[t]);
    }
    uint64_t bad = 0;
    *first_bad = 0;
    for (int t = 0; t < nthreads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].bad && bad == 0) *first_bad = jobs[t].first_bad;
        bad += jobs[t].bad;
    }
    return bad;
}

/* ------------------------------------------------------------------------- */
/* amax, scale, quantize.                                                      */
/* ------------------------------------------------------------------------- */

/* Scale from amax: s = fl32(fmax / amax), d = fl32(1 / s), both IEEE
 * correctly rounded FP32 divisions.  When amax is zero, not finite, or gives
 * a scale that is zero or not finite (as does the inverse), both are 1. */
void orc_scale(int fmt, float amax, float *s_out, float *d_out)
{
    volatile float fmax = (float)orc_max_finite(fmt);
    volatile float s = fmax / amax;
    volatile float d = 1.0f / s;
    if (!(amax > 0.0f) || !isfinite(amax) || !isfinite(s) || s == 0.0f || !isfinite(d)) {
        s = 1.0f;
        d = 1.0f;
    }
    *s_out = s;
    *d_out = d;
}

/* amax = max |x| over the tensor (per_row = 0) or over each row (per_row = 1).
 * A NaN anywhere makes that amax NaN.  Then q = enc(fl32(x * s)).
 * Row-major rows x cols input with leading dimension ldx; codes go to q with
 * leading dimension ldq; s and d receive 1 or rows floats. */
void orc_quantize(const float *x, int64_t rows, int64_t cols, int64_t ldx, int fmt, int per_row,
                  uint8_t *q, int64_t ldq, float *s, float *d)
{
    float tensor_amax = 0.0f;
    if (!per_row) {
        for (int64_t r = 0; r < rows; ++r)
            for (int64_t c = 0; c < cols; ++c) {
                float v = fabsf(x[r * ldx + c]);
                if (isnan(v) || isnan(tensor_amax)) tensor_amax = NAN;
                else if (v > tensor_amax) tensor_amax = v;
            }
        orc_scale(fmt, tensor_amax, &s[0], &d[0]);
    }
    for (int64_t r = 0; r < rows; ++r) {
        float sr;
        if (per_row) {
            float amax = 0.0f;
            for (int64_t c = 0; c < cols; ++c) {
                float v = fabsf(x[r * ldx + c]);
                if (isnan(v) || isnan(amax)) amax = NAN;
                else if (v > amax) amax = v;
            }
            orc_scale(fmt, amax, &s[r], &d[r]);
            sr = s[r];
        } else {
            sr = s[0];
        }
        for (int64_t c = 0; c < cols; ++c) {
            volatile float y = x[r * ldx + c] * sr;   /* one FP32 product, then encode */
            q[r * ldq + c] = orc_encode(fmt, y);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* 2:4 pruning and the compressed format.                                      */
/* ------------------------------------------------------------------------- */

/* Order used to choose survivors: larger magnitude first, then lower index.
 * For finite codes magnitude is |decode|.  NaN and infinity codes are ranked
 * by their 7-bit magnitude field, which puts them above every finite code. */
static int ranks_above(int fmt, uint8_t a, int ia, uint8_t b, int ib)
{
    double va = orc_decode(fmt, a), vb = orc_decode(fmt, b);
    int cmp;
    if (isfinite(va) && isfinite(vb)) {
        double ma = fabs(va), mb = fabs(vb);
        cmp = ma > mb ? 1 : (ma < mb ? -1 : 0);
    } else {
        int ka = a & 0x7F, kb = b & 0x7F;
        cmp = ka > kb ? 1 : (ka < kb ? -1 : 0);
    }
    if (cmp != 0) return cmp > 0;
    return ia < ib;
}

/* Prune a row-major rows x K code matrix (K % 4 == 0) to 2:4 along K and
 * compress it.  Rule, per row r and group g (k = 4g .. 4g+3): order the four
 * indices by (magnitude descending, index ascending) and keep the first two;
 * the survivors are stored in ascending index order.
 *   values[r*(K/2) + 2g + t] = code of the t-th survivor (t = 0, 1)
 *   meta[r*(K/8) + g/2]      nibble (g % 2) (low nibble for even g) = i0 | i1 << 2,
 *                            i0 < i1 the survivor positions within the group
 *   mask[r*(K/8) + k/8]      bit (k % 8) set iff element k survives   (mask may be NULL)
 *   pruned[r*K + k]          the input code if it survives, else +0 (0x00)  (may be NULL) */
void orc_prune24(const uint8_t *x, int fmt, int64_t rows, int64_t K, int64_t ldx,
                 uint8_t *values, uint8_t *meta, uint8_t *mask, uint8_t *pruned)
{
    for (int64_t r = 0; r < rows; ++r) {
        const uint8_t *row = x + r * ldx;
        for (int64_t g = 0; g < K / 4; ++g) {
            const uint8_t *c = row + 4 * g;
            /* rank of each index = number of indices that rank above it */
            int keep[4];
            for (int i = 0; i < 4; ++i) {
                int above = 0;
                for (int j = 0; j < 4; ++j)
                    if (j != i && ranks_above(fmt, c[j], j, c[i], i)) above++;
                keep[i] = above < 2;
            }
            int pos[2], n = 0;
            for (int i = 0; i < 4; ++i)
                if (keep[i]) pos[n++] = i;
            values[r * (K / 2) + 2 * g + 0] = c[pos[0]];
            values[r * (K / 2) + 2 * g + 1] = c[pos[1]];
            uint8_t nib = (uint8_t)(pos[0] | (pos[1] << 2));
            uint8_t *mb = &meta[r * (K / 8) + g / 2];
            if (g % 2 == 0) *mb = (uint8_t)((*mb & 0xF0) | nib);
            else *mb = (uint8_t)((*mb & 0x0F) | (nib << 4));
            for (int i = 0; i < 4; ++i) {
                int64_t k = 4 * g + i;
                if (mask) {
                    uint8_t *bb = &mask[r * (K / 8) + k / 8];
                    if (keep[i]) *bb = (uint8_t)(*bb | (1u << (k % 8)));
                    else *bb = (uint8_t)(*bb & ~(1u << (k % 8)));
                }
                if (pruned) pruned[r * K + k] = keep[i] ? c[i] : 0x00;
            }
        }
    }
}

/* Inverse of the compression: a dense rows x K code matrix with +0 (0x00) at
 * the dropped positions. */
void orc_decompress24(const uint8_t *values, const uint8_t *meta, int64_t rows, int64_t K, uint8_t *out)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t g = 0; g < K / 4; ++g) {
            uint8_t mb = meta[r * (K / 8) + g / 2];
            uint8_t nib = (g % 2 == 0) ? (mb & 0xF) : (mb >> 4);
            int i0 = nib & 3, i1 = (nib >> 2) & 3;
            for (int i = 0; i < 4; ++i) out[r * K + 4 * g + i] = 0x00;
            out[r * K + 4 * g + i0] = values[r * (K / 2) + 2 * g + 0];
            out[r * K + 4 * g + i1] = values[r * (K / 2) + 2 * g + 1];
        }
}

/* ------------------------------------------------------------------------- */
/* GEMM in FP64.                                                               */
/* ------------------------------------------------------------------------- */

/* C_ref[i,j] = d_a[i] * d_b[j] * sum_k dec(A[i,k]) * dec(B[k,j])
 * S_abs[i,j] = |d_a[i] * d_b[j]| * sum_k |dec(A[i,k]) * dec(B[k,j])|
 * A: row-major M x K codes (lda); B: column-major K x N codes, i.e. N rows of
 * K codes (ldb).  d_a has M entries if a_per_row else 1; d_b has N entries if
 * b_per_col else 1.  For E4M3 x E4M3 every partial sum is a multiple of 2^-18
 * below 2^32 when K <= 16384, so the FP64 sum is exact and its order does not
 * matter. */
typedef struct {
    const uint8_t *a; int a_fmt; int64_t lda;
    const uint8_t *b; int b_fmt; int64_t ldb;
    const float *da; int a_per_row;
    const float *db; int b_per_col;
    int64_t M, N, K;
    double *cref, *sabs;           /* row-major M x N, leading dimension N */
    int64_t row_lo, row_hi;
    double lut_a[256], lut_b[256];
} gemm_job;

static void gemm_entry(const gemm_job *j, int64_t i, int64_t jj, const double *arow, double *c, double *s)
{
    const uint8_t *bcol = j->b + jj * j->ldb;
    double sum = 0.0, asum = 0.0;
    for (int64_t k = 0; k < j->K; ++k) {
        double p = arow[k] * j->lut_b[bcol[k]];
        sum += p;
        asum += fabs(p);
    }
    double da = j->da[j->a_per_row ? i : 0], db = j->db[j->b_per_col ? jj : 0];
    *c = (sum * da) * db;
    *s = fabs(da * db) * asum;
}

static void *gemm_worker(void *p)
{
    gemm_job *j = (gemm_job *)p;
    double *arow = (double *)malloc(sizeof(double) * (size_t)(j->K > 0 ? j->K : 1));
    for (int64_t i = j->row_lo; i < j->row_hi; ++i) {
        for (int64_t k = 0; k < j->K; ++k) arow[k] = j->lut_a[j->a[i * j->lda + k]];
        for (int64_t jj = 0; jj < j->N; ++jj)
            gemm_entry(j, i, jj, arow, &j->cref[i * j->N + jj], &j->sabs[i * j->N + jj]);
    }
    free(arow);
    return NULL;
}

static void fill_luts(gemm_job *j)
{
    for (int c = 0; c < 256; ++c) {
        j->lut_a[c] = orc_decode(j->a_fmt, (uint8_t)c);
        j->lut_b[c] = orc_decode(j->b_fmt, (uint8_t)c);
    }
}

/* Full M x N result for rows [row_lo, row_hi) (pass 0, M for all rows), on
 * nthreads threads that each take a contiguous block of rows.  cref and sabs
 * are indexed by the absolute row. */
void orc_gemm(const uint8_t *a, int a_fmt, int64_t lda, const uint8_t *b, int b_fmt, int64_t ldb,
              const float *da, int a_per_row, const float *db, int b_per_col,
              int64_t M, int64_t N, int64_t K, int64_t row_lo, int64_t row_hi,
              double *cref, double *sabs, int nthreads)
{
    (void)M;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    gemm_job *jobs = (gemm_job *)calloc((size_t)nthreads, sizeof(gemm_job));
    pthread_t th[256];
    int64_t rows = row_hi - row_lo, step = (rows + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        gemm_job *j = &jobs[t];
        j->a = a; j->a_fmt = a_fmt; j->lda = lda;
        j->b = b; j->b_fmt = b_fmt; j->ldb = ldb;
        j->da = da; j->a_per_row = a_per_row; j->db = db; j->b_per_col = b_per_col;
        j->M = M; j->N = N; j->K = K; j->cref = cref; j->sabs = sabs;
        j->row_lo = row_lo + step * t < row_hi ? row_lo + step * t : row_hi;
        j->row_hi = row_lo + step * (t + 1) < row_hi ? row_lo + step * (t + 1) : row_hi;
        fill_luts(j);
        pthread_create(&th[t], NULL, gemm_worker, j);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(jobs);
}

/* The same entries, one by one, at the listed (i, j) positions: used to check
 * full-size GPU results on a sample of outputs. */
void orc_gemm_at(const uint8_t *a, int a_fmt, int64_t lda, const uint8_t *b, int b_fmt, int64_t ldb,
                 const float *da, int a_per_row, const float *db, int b_per_col, int64_t K,
                 const int64_t *ii, const int64_t *jj, int64_t n, double *cref, double *sabs)
{
    gemm_job *j = (gemm_job *)calloc(1, sizeof(gemm_job));
    j->a = a; j->a_fmt = a_fmt; j->lda = lda;
    j->b = b; j->b_fmt = b_fmt; j->ldb = ldb;
    j->da = da; j->a_per_row = a_per_row; j->db = db; j->b_per_col = b_per_col;
    j->K = K;
    fill_luts(j);
    double *arow = (double *)malloc(sizeof(double) * (size_t)(K > 0 ? K : 1));
    for (int64_t t = 0; t < n; ++t) {
        for (int64_t k = 0; k < K; ++k) arow[k] = j->lut_a[a[ii[t] * lda + k]];
        gemm_entry(j, ii[t], jj[t], arow, &cref[t], &sabs[t]);
    }
    free(arow);
    free(j);
}

/* ------------------------------------------------------------------------- */
/* GEMM of real-valued operands in FP64 (the FP32 / FP16 / BF16 stages).       */
/* ------------------------------------------------------------------------- */

/* The mixed-precision sequence of Sec. 8.3 runs FP32 and 16-bit GEMM stages
 * beside the FP8 one.  Their definition, with a and b the exact FP64 values
 * of the stage's FP32, FP16 or BF16 inputs:
 *   C_ref[i,j] = s_a[i] * s_b[j] * sum_k a[i,k] * b[j,k]
 *   S_abs[i,j] = |s_a[i] * s_b[j]| * sum_k |a[i,k] * b[j,k]|
 * a: row-major M x K (lda); b: N rows of K (ldb), i.e. B column-major; s_a
 * has M entries if a_per_row else 1, s_b N entries if b_per_col else 1.  A
 * product of two such values has at most 48 significant bits and is exact
 * in FP64; the FP64 sum (k ascending) errs by at most K 2^-53 S_abs, a
 * 2^-29 fraction of the acceptance bound 4 K 2^-24 S_abs. */
typedef struct {
    const double *a; int64_t lda;
    const double *b; int64_t ldb;
    const float *sa; int a_per_row;
    const float *sb; int b_per_col;
    int64_t N, K;
    double *cref, *sabs;
    int64_t row_lo, row_hi;
} real_job;

static void *real_worker(void *p)
{
    real_job *j = (real_job *)p;
    for (int64_t i = j->row_lo; i < j->row_hi; ++i) {
        for (int64_t jj = 0; jj < j->N; ++jj) {
            double sum = 0.0, asum = 0.0;
            for (int64_t k = 0; k < j->K; ++k) {
                double prod = j->a[i * j->lda + k] * j->b[jj * j->ldb + k];
                sum += prod;
                asum += fabs(prod);
            }
            double sa = j->sa[j->a_per_row ? i : 0], sb = j->sb[j->b_per_col ? jj : 0];
            j->cref[i * j->N + jj] = (sum * sa) * sb;
            j->sabs[i * j->N + jj] = fabs(sa * sb) * asum;
        }
    }
    return NULL;
}

void orc_gemm_real(const double *a, int64_t lda, const double *b, int64_t ldb, const float *sa, int a_per_row,
                   const float *sb, int b_per_col, int64_t M, int64_t N, int64_t K, double *cref, double *sabs,
                   int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    real_job jobs[256];
    pthread_t th[256];
    int64_t step = (M + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        real_job *j = &jobs[t];
        j->a = a; j->lda = lda; j->b = b; j->ldb = ldb;
        j->sa = sa; j->a_per_row = a_per_row; j->sb = sb; j->b_per_col = b_per_col;
        j->N = N; j->K = K; j->cref = cref; j->sabs = sabs;
        j->row_lo = step * t < M ? step * t : M;
        j->row_hi = step * (t + 1) < M ? step * (t + 1) : M;
        pthread_create(&th[t], NULL, real_worker, j);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------- */
/* Batch encode of consecutive FP32 bit patterns (for exhaustive checks).      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int fmt;
    uint32_t lo;
    int64_t begin, end;
    uint8_t *out;
} range_job;

static void *range_worker(void *p)
{
    range_job *j = (range_job *)p;
    for (int64_t t = j->begin; t < j->end; ++t) {
        uint32_t b = j->lo + (uint32_t)t;
        float x;
        memcpy(&x, &b, 4);
        j->out[t] = orc_encode(j->fmt, x);
    }
    return NULL;
}

/* out[t] = orc_encode(fmt, the float whose bits are lo + t), t < n. */
void orc_encode_range(int fmt, uint32_t lo, int64_t n, uint8_t *out, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    range_job jobs[256];
    int64_t step = (n + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fmt = fmt;
        jobs[t].lo = lo;
        jobs[t].begin = step * t < n ? step * t : n;
        jobs[t].end = step * (t + 1) < n ? step * (t + 1) : n;
        jobs[t].out = out;
        pthread_create(&th[t], NULL, range_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}
