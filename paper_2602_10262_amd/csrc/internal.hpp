// Host-side declarations shared by the kernel files and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fp8k {

constexpr int kBKHost = 128;   // K step of every GEMM kernel (codes)

// One GEMM as the kernels see it.  The "i" operand sits in the MFMA A slot
// (dense rows, or 2:4-compressed values + metadata when sparse), the "j"
// operand in the MFMA B slot (dense rows of K codes, or 2:4-compressed rows
// that the kernel expands to dense ones on their way into LDS).  The result
// element (i, j) is stored at c[i*ldc + j], or at c[j*ldc + i] when
// trans_out is set (used when the compressed operand is the weight).
struct GemmParams {
    const uint8_t *a;      // i operand: dense M x K (lda) or compressed values M x K/2 (lda)
    const uint8_t *meta;   // i operand metadata M x K/8 (ldm) when sparse
    const uint8_t *b;      // j operand: N x K (ldb), or compressed values N x K/2 when meta_b is set
    const uint8_t *meta_b; // j operand metadata N x K/8 (ldmb) when both operands are 2:4-compressed
    const float *si;       // descale of row i (or one for all rows)
    const float *sj;       // descale of column j (or one)
    void *c;
    float *ws;             // split-K partial sums [splits][M][N] when splits > 1
    int64_t lda, ldm, ldb, ldc, ldmb;
    int M, N, K;
    int si_per, sj_per;    // 1: one descale per row / column
    int out_bf16;          // BF16 output (RNE)
    int out_f16;           // FP16 output (RNE); neither: FP32
    int trans_out;         // store transposed; descales then apply j first
    int splits;            // >= 1
    int kchunk;            // K range per split, a multiple of 128
};

struct TileDesc {
    int bm, bn, waves, sparse_ok;
    int exact;     // FP8 decoded to BF16 and summed on the BF16 MFMA (bound holds for every K)
    int dense_ok;  // has a dense kernel (a 2:4-only tile's dense stages would not fit in LDS)
};

// Below this K the FP8 MFMA's in-instruction truncation is not guaranteed to
// stay inside 4 K 2^-24 sum |a b| (its error reaches about 7 2^-13 of the
// largest product of each run of eight k), so plans the library chooses use
// the exact-sum tiles there.
constexpr int kExactBelowK = 3584;

int num_tiles();
const TileDesc &tile_desc(int t);

// Whether K avoids partial 16-byte chunks; otherwise launch_gemm uses the
// 128 x 128 byte-exact kernel whatever the tile.
bool k_is_fast(bool sparse, int K);
hipError_t launch_gemm(int tile, int fa, int fb, bool sparse, const GemmParams &p, hipStream_t st);
hipError_t launch_splitk_reduce(const GemmParams &p, hipStream_t st);
// Both operands compressed (p.meta and p.meta_b set): tiles that have such a
// kernel, and its launch.
bool both_tile_supported(int tile);
hipError_t launch_gemm_both(int tile, int fa, int fb, const GemmParams &p, hipStream_t st);

hipError_t launch_quantize(const float *x, int64_t rows, int64_t cols, int64_t ldx, int fmt, int per_row,
                           uint8_t *q, int64_t ldq, float *s, float *d, void *ws, hipStream_t st);
// Clears *amax_bits and reduces max |x| (FP32 bit pattern) into it.
hipError_t launch_amax_tensor(const float *x, int64_t rows, int64_t cols, int64_t ldx, uint32_t *amax_bits,
                              hipStream_t st);
// Quantize (per tensor or per row) and 2:4 prune/compress in one pass; ws
// holds the amax word of the per-tensor form.
hipError_t launch_quantize_prune24(const float *x, int64_t rows, int64_t K, int64_t ldx, int fmt, int per_row,
                                   uint8_t *values, uint8_t *meta, uint8_t *mask, float *s, float *d, void *ws,
                                   hipStream_t st);
hipError_t launch_encode_bits(int fmt, uint32_t lo, int64_t n, uint8_t *out, hipStream_t st);

hipError_t launch_prune24(const uint8_t *x, int64_t rows, int64_t K, int64_t ldx, uint8_t *values,
                          uint8_t *meta, uint8_t *mask, hipStream_t st);
hipError_t launch_decompress24(const uint8_t *values, const uint8_t *meta, int64_t rows, int64_t K,
                               uint8_t *out, int64_t ldo, hipStream_t st);

hipError_t launch_validate(const void *c, int out_bf16, int64_t ldc, const double *cref, const double *sabs,
                           int64_t M, int64_t N, int64_t K, double *out, hipStream_t st);

// Grouped persistent GEMM.
struct GroupEntry {
    GemmParams p;          // splits == 1
    int sparse;
    int tiles_m, tiles_n;
    int64_t tile_begin;    // prefix sum of tiles over the work list
};
int grouped_max_workgroups(int tile);
bool grouped_tile_supported(int tile);

}  // namespace fp8k
