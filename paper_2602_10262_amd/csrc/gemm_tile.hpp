// The FP8 GEMM macro-tile shared by the plain, split-K and grouped kernels.
//
// One workgroup computes a BM x BN block of C over a K range, in steps of 128
// codes of K.  The pipelines (PF in the tile table, see gemm_tile):
//   - register-staged (PF 1-3): 128-bit global loads of a later step go to
//     registers before the MFMAs of the current one and are written to the
//     other half of a double-buffered LDS area after them;
//   - LDS-DMA ring (PF >= 6): buffer loads straight into LDS, NS stages, one
//     loader wave per SIMD when a workgroup has two per SIMD;
//   - exact sums (PF 40 through registers, 42-44 on the DMA ring): FP8 codes
//     decoded exactly to BF16 and summed on the BF16 MFMA, for K below 3584;
//   - 32 x 32 x 64 MFMAs on the DMA ring (PF 56);
//   - FP32 / FP16 / BF16 operands on the DMA ring (the HP parameter).
// LDS layout: dense operands keep one 128-byte row per tile row, the
// sixteen-byte chunks of row r permuted by an XOR with the row number so that
// the rows a fragment read touches spread over all banks; compressed operands
// keep 64 value bytes and 16 metadata bytes per row.  Each wave owns a
// (BM / WM) x (BN / WN) sub-block made of 16 x 16 accumulators; per step it
// reads its A and B fragments from LDS and issues v_mfma_f32_16x16x128_f8f6f4
// (dense: lane l supplies row l % 16, codes 32 (l / 16) .. 32 (l / 16) + 31 of
// the step, for both operands) or v_smfmac_f32_16x16x128_* (2:4: lane l
// supplies the 16 survivors of those 32 positions and their eight index
// nibbles as one 32-bit word, while its B lane holds codes 16 (l / 16) + 0..15
// and 64 + 16 (l / 16) + 0..15, the layout the sparse instruction pairs with).
// Epilogue: descales applied in FP32, C stored as FP32, BF16 or FP16 (RNE), or
// raw FP32 partial sums to the split-K workspace.
#pragma once
#include <type_traits>
#include "common.hpp"
#include "internal.hpp"

namespace fp8k {

constexpr int kBK = 128;
// Pipeline number of the exact-sum tiles (FP8 decoded to BF16, BF16 MFMA).
constexpr int kExactPF = 40;
// Pipelines kExactPF + 2 .. kExactPF + 4: exact sums on the LDS-DMA ring with
// PF - kExactPF stages of FP8 codes (a 2:4 operand compressed), decoded (and
// expanded) after the fragment reads; K a multiple of 16 (128 with a 2:4
// operand), any other K runs on kExactAnyKTile.
constexpr bool pf_exact_dma(int pf) { return pf >= kExactPF + 2 && pf <= kExactPF + 4; }
constexpr bool pf_exact(int pf) { return pf == kExactPF || pf_exact_dma(pf); }
constexpr int kExactAnyKTile = 27;
// Pipelines 56 .. 58: the FP8 LDS-DMA ring with PF - 54 stages on the
// 32 x 32 x 64 MFMA instead of the 16 x 16 x 128 one (dense operands).
constexpr bool pf_mfma32(int pf) { return pf >= 56 && pf <= 58; }
// Operand types of the higher-precision GEMMs (the DMA ring's HP parameter;
// -1 there means FP8 codes).
constexpr int kHpF32 = 0, kHpF16 = 1, kHpBF16 = 2;
// Buffer resource word 3 for raw (unswizzled, unformatted) dword access on gfx9.
constexpr int kBufferFlags = 0x00020000;

template <int V>
struct Int {
    static constexpr int value = V;
};

// Calls f(Int<I>{}) for I = B .. E-1 with compile-time indices (keeps arrays
// indexed by them in registers whatever the unroller decides).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(Int<B>{});
        static_for<B + 1, E>(f);
    }
}

// Tile table: (BM, BN, WM, WN, workgroups per CU the registers are sized
// for, pipeline PF as described at gemm_tile).  Index = plan.tile.
#define FP8_TILE_LIST(X)           \
    X(0, 128, 128, 2, 2, 2, 2)     \
    X(1, 256, 128, 2, 2, 1, 2)     \
    X(2, 256, 256, 2, 2, 1, 1)     \
    X(3, 64, 64, 1, 1, 8, 2)       \
    X(4, 16, 64, 1, 1, 8, 2)       \
    X(5, 32, 128, 1, 2, 4, 2)      \
    X(6, 128, 256, 2, 2, 1, 2)     \
    X(7, 64, 256, 1, 4, 2, 2)      \
    X(8, 128, 16, 4, 1, 2, 2)      \
    X(9, 256, 32, 4, 1, 2, 2)      \
    X(10, 256, 256, 2, 4, 1, 1)    \
    X(11, 256, 256, 4, 2, 1, 2)    \
    X(12, 256, 128, 4, 2, 1, 2)    \
    X(13, 128, 256, 2, 4, 1, 2)    \
    X(14, 128, 256, 2, 4, 1, 3)    \
    X(15, 256, 128, 4, 2, 1, 3)    \
    X(16, 128, 128, 2, 2, 1, 3)    \
    X(17, 256, 128, 2, 2, 1, 7)    \
    X(18, 128, 256, 2, 2, 1, 7)    \
    X(19, 256, 256, 2, 4, 1, 6)    \
    X(20, 16, 256, 1, 4, 1, 8)     \
    X(21, 32, 256, 1, 4, 1, 8)     \
    X(22, 64, 256, 1, 4, 1, 7)     \
    X(23, 128, 256, 2, 4, 1, 7)    \
    X(24, 16, 32, 1, 1, 2, 16)     \
    X(25, 128, 128, 2, 2, 1, 40)   \
    X(26, 64, 64, 2, 2, 2, 40)     \
    X(27, 128, 128, 2, 4, 1, 40)   \
    X(28, 128, 128, 2, 4, 1, 44)   \
    X(29, 256, 128, 4, 2, 1, 43)   \
    X(30, 256, 256, 2, 4, 1, 42)   \
    X(31, 256, 256, 2, 4, 1, 56)


// Whether a tile of BM rows has a 2:4 kernel: its compressed rows fill whole
// 1 KiB DMA blocks of metadata (BM % 64 == 0), or fit the register pipeline's
// single round of loads (BM <= 32).
constexpr bool tile_sparse_ok(int bm) { return bm % 64 == 0 || bm <= 32; }

constexpr int kMaxLdsBytes = 160 * 1024;   // LDS of one CU (gfx950)

// Stages of pipeline pf: 2 for the register-prefetch loops, 3 for the loop
// that also prefetches fragments, PF - 4 for the DMA loops, PF - kExactPF for
// the exact-sum DMA loops.
constexpr int pf_stages(int pf)
{
    return pf == 3 ? 3
                   : (pf == kExactPF ? 2
                                     : (pf_exact_dma(pf) ? pf - kExactPF
                                                         : (pf_mfma32(pf) ? pf - 54 : (pf >= 6 ? pf - 4 : 2))));
}

// LDS of one tile: NSTAGE stages.
template <int BM, int BN, bool SP, int PF = 2>
struct TileSmem {
    // the exact-sum pipeline (PF == kExactPF) keeps both operands as BF16,
    // a 2:4 operand already expanded to its dense rows
    static constexpr bool EXACT = PF == kExactPF;
    static constexpr int A_BYTES = EXACT ? BM * 256 : (SP ? BM * 64 : BM * 128);
    static constexpr int M_BYTES = (SP && !EXACT) ? BM * 16 : 0;
    static constexpr int B_BYTES = EXACT ? BN * 256 : BN * 128;
    static constexpr int STAGE = A_BYTES + M_BYTES + B_BYTES;
    static constexpr int NSTAGE = pf_stages(PF);
    static constexpr int TOTAL = NSTAGE * STAGE;
};

// Whether a tile's dense / 2:4 kernel fits in LDS (a three-stage 256 x 256
// ring fits only with the compressed operand: 3 x 52 KiB).
constexpr bool tile_dense_fits(int bm, int bn, int pf)
{
    return pf_stages(pf) * ((pf == kExactPF ? 256 : 128) * (bm + bn)) <= kMaxLdsBytes;
}

// LDS swizzles.  Each is checked on the GPU with the LDS microbenchmarks
// (fp8_ubench_lds_pattern, and fp8_ubench_lds_offsets over the 256 swizzles
// that XOR row bits into the chunk index): a fragment read of 16 rows x 4
// chunk positions must take the 4 LDS cycles of a conflict-free 128-bit read,
// not 8.

// Compressed rows (64 value bytes) keep their 16-byte chunk c at c ^ h(r),
// h(r) = ((r >> 1) & 1) ^ (((r >> 3) & 1) << 1).  (The earlier
// ((r >> 1) & 3) ^ ((r >> 3) & 1), and the unswizzled layout, cost 8 cycles.)
__device__ __forceinline__ int swz_sp(int r, int c)
{
    return r * 64 + ((c ^ ((r >> 1) & 1) ^ (((r >> 3) & 1) << 1)) << 4);
}

// Dense rows (128 bytes) of the dense kernels: chunk c of row r sits at
// c ^ g(r), g(r) = (r & 7) ^ ((r >> 3) & 1); the dense fragment reads chunk
// positions (2g, 2g + 1) in two conflict-free instructions.
__device__ __forceinline__ int swz(int r, int c) { return (r * 128) + ((c ^ (r & 7) ^ ((r >> 3) & 1)) << 4); }

// Dense B rows of the 2:4 kernels: the 2:4 instruction reads chunk
// positions (g, g + 4) instead of (2g, 2g + 1), which g(r) serves in 8
// cycles; g2(r) = (r & 7) ^ (((r >> 3) & 1) << 1) serves them in 4.
__device__ __forceinline__ int swz_b2(int r, int c)
{
    return (r * 128) + ((c ^ (r & 7) ^ (((r >> 3) & 1) << 1)) << 4);
}
// B-row swizzle of a kernel: SP (2:4 kernels) or dense.
template <bool SP>
__device__ __forceinline__ int swz_b(int r, int c) { return SP ? swz_b2(r, c) : swz(r, c); }

// 16 bytes from global memory; `valid` (0..16) leading bytes are real, the
// rest take `fill`.
__device__ __forceinline__ uint4 load16_partial(const uint8_t *p, int valid, uint32_t fill)
{
    uint32_t w[4] = {fill, fill, fill, fill};
    for (int b = 0; b < valid && b < 16; ++b) {
        w[b / 4] &= ~(0xFFu << (8 * (b % 4)));
        w[b / 4] |= (uint32_t)p[b] << (8 * (b % 4));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <int FA, int FB>
__device__ __forceinline__ v4f mfma_dense(const v8i &a, const v8i &b, const v4f &c)
{
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, FA, FB, 0, 0, 0, 0);
}

template <int FA, int FB>
__device__ __forceinline__ v4f mfma_sparse(const v4i &a, const v8i &b, const v4f &c, int idx)
{
    if constexpr (FA == kE4M3 && FB == kE4M3) return __builtin_amdgcn_smfmac_f32_16x16x128_fp8_fp8(a, b, c, idx, 0, 0);
    else if constexpr (FA == kE5M2 && FB == kE4M3) return __builtin_amdgcn_smfmac_f32_16x16x128_bf8_fp8(a, b, c, idx, 0, 0);
    else if constexpr (FA == kE4M3 && FB == kE5M2) return __builtin_amdgcn_smfmac_f32_16x16x128_fp8_bf8(a, b, c, idx, 0, 0);
    else return __builtin_amdgcn_smfmac_f32_16x16x128_bf8_bf8(a, b, c, idx, 0, 0);
}

__device__ __forceinline__ void store_out(const GemmParams &p, int i, int j, float acc)
{
    float si = p.si[p.si_per ? i : 0], sj = p.sj[p.sj_per ? j : 0];
    float v = p.trans_out ? (acc * sj) * si : (acc * si) * sj;
    int64_t off = p.trans_out ? (int64_t)j * p.ldc + i : (int64_t)i * p.ldc + j;
    if (p.out_bf16) reinterpret_cast<uint16_t *>(p.c)[off] = f32_to_bf16_rne(v);
    else if (p.out_f16) reinterpret_cast<uint16_t *>(p.c)[off] = f32_to_f16_rne(v);
    else reinterpret_cast<float *>(p.c)[off] = v;
}

// Stores the four accumulator values of a lane: (i, j + q) when ALONG_J,
// else (i + q, j), q = 0..3; to the split-K workspace when splits > 1.
template <bool ALONG_J>
__device__ __forceinline__ void store4(const GemmParams &p, int i, int j, int split, const v4f &v)
{
    if (p.splits > 1) {
        float *w = p.ws + (int64_t)split * p.M * p.N;
        if (ALONG_J) {
            if (i >= p.M) return;
            if (j + 3 < p.N && (p.N % 4) == 0) {
                *reinterpret_cast<float4 *>(w + (int64_t)i * p.N + j) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                for (int q = 0; q < 4; ++q)
                    if (j + q < p.N) w[(int64_t)i * p.N + j + q] = v[q];
            }
        } else {
            if (j >= p.N) return;
            for (int q = 0; q < 4; ++q)
                if (i + q < p.M) w[(int64_t)(i + q) * p.N + j] = v[q];
        }
        return;
    }
    // Output columns are consecutive for (ALONG_J, not transposed) and for
    // (along i, transposed).
    const bool contiguous = ALONG_J ? !p.trans_out : p.trans_out;
    const int row = ALONG_J ? (p.trans_out ? j : i) : (p.trans_out ? j : i);
    const int col0 = ALONG_J ? (p.trans_out ? i : j) : (p.trans_out ? i : j);
    if (contiguous) {
        const int rows = p.trans_out ? p.N : p.M, cols = p.trans_out ? p.M : p.N;
        if (row >= rows) return;
        float o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int iq = ALONG_J ? i : i + q, jq = ALONG_J ? j + q : j;
            const float si = p.si[p.si_per ? min(iq, p.M - 1) : 0], sj = p.sj[p.sj_per ? min(jq, p.N - 1) : 0];
            o[q] = p.trans_out ? (v[q] * sj) * si : (v[q] * si) * sj;
        }
        const int64_t off = (int64_t)row * p.ldc + col0;
        const bool vec = col0 + 3 < cols && (p.ldc % 4) == 0 && ((reinterpret_cast<uintptr_t>(p.c) & 15) == 0);
        if (p.out_bf16 || p.out_f16) {
            uint16_t *c = reinterpret_cast<uint16_t *>(p.c) + off;
            uint16_t h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) h[q] = p.out_bf16 ? f32_to_bf16_rne(o[q]) : f32_to_f16_rne(o[q]);
            if (vec) {
                uint2 w;
                w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
                w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
                *reinterpret_cast<uint2 *>(c) = w;
            } else {
                for (int q = 0; q < 4; ++q)
                    if (col0 + q < cols) c[q] = h[q];
            }
        } else {
            float *c = reinterpret_cast<float *>(p.c) + off;
            if (vec) *reinterpret_cast<float4 *>(c) = make_float4(o[0], o[1], o[2], o[3]);
            else
                for (int q = 0; q < 4; ++q)
                    if (col0 + q < cols) c[q] = o[q];
        }
    } else {
        for (int q = 0; q < 4; ++q) {
            const int iq = ALONG_J ? i : i + q, jq = ALONG_J ? j + q : j;
            if (iq < p.M && jq < p.N) store_out(p, iq, jq, v[q]);
        }
    }
}

// Orders a wave's LDS accesses across lanes without a workgroup barrier:
// the instructions of one wave reach the LDS in program order, so only the
// compiler has to be kept from moving accesses across this point (the
// fences at wavefront scope) and the wave's own LDS operations must have
// completed.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The staged store of write_tile for one output orientation: TR = the
// result is stored transposed (output rows are j).  Pass t covers the
// sixteen output rows of MFMA block t along the output-row index.  The
// descales a lane needs are loaded once, before the workgroup barrier, so
// their latency overlaps it: the row descales of every pass, and the column
// descales of the one 16-byte column chunk the lane stores in every row.
template <int BM, int BN, int WM, int WN, bool ALONG_J, int LDS_BYTES, bool TR>
__device__ __forceinline__ void write_tile_staged(const GemmParams &p, const v4f (&acc)[BM / WM / 16][BN / WN / 16],
                                                  int m0, int n0, int wave, int lane, uint8_t *smem)
{
    constexpr int NW = WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    constexpr int STRIDE = (WTN > WTM ? WTN : WTM) * 4 + 16;   // padded FP32 staging row (bytes)
    static_assert(NW * 16 * STRIDE <= LDS_BYTES, "epilogue staging exceeds the tile's LDS");
    constexpr int NPASS = TR ? TN : TM;
    constexpr int OC = TR ? WTM : WTN;                          // output columns of this wave
    constexpr bool ROW_PER_Q = TR ? ALONG_J : !ALONG_J;         // the four values sit in four output rows
    constexpr int RQ = ROW_PER_Q ? 4 : 1;
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lg = lane >> 4;
    const bool bf = p.out_bf16 != 0 || p.out_f16 != 0;   // 16-bit output
    const bool f16 = p.out_f16 != 0 && p.out_bf16 == 0;
    const int esz = bf ? 2 : 4;
    const int per = bf ? 8 : 4;                                 // output elements per 16-byte chunk
    const int chunks_row = OC / per;                            // divides 64: a lane's chunk column is fixed
    uint8_t *reg = smem + wave * 16 * STRIDE;
    const int rows_out = TR ? p.N : p.M, cols_out = TR ? p.M : p.N;
    const int orow0 = TR ? n0 + wn * WTN : m0 + wm * WTM;       // wave's first output row
    const int ocol0 = TR ? m0 + wm * WTM : n0 + wn * WTN;       // wave's first output column
    const float *rdesc = TR ? p.sj : p.si, *cdesc = TR ? p.si : p.sj;
    const int rper = TR ? p.sj_per : p.si_per, cper = TR ? p.si_per : p.sj_per;
    const bool vec_ok = ((p.ldc * esz) % 16) == 0 && ((reinterpret_cast<uintptr_t>(p.c) & 15) == 0);
    const int cc = lane % chunks_row, rsub = lane / chunks_row, rstep = 64 / chunks_row;
    const int ocol = ocol0 + cc * per;
    float rd[NPASS][RQ], cd[8];
    static_for<0, NPASS>([&](auto tt) {
        constexpr int t = decltype(tt)::value;
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const int orow = min(orow0 + t * 16 + (ROW_PER_Q ? 4 * lg + q : lr), rows_out - 1);
            rd[t][q] = rdesc[rper ? orow : 0];
        }
    });
#pragma unroll
    for (int e = 0; e < 8; ++e) cd[e] = cdesc[cper ? min(ocol + e, cols_out - 1) : 0];
    __syncthreads();   // every wave is done with the main loop's LDS
    static_for<0, NPASS>([&](auto tt) {
        constexpr int t = decltype(tt)::value;
        // stage the pass's accumulators times their output row's descale
        if constexpr (!TR) {
            static_for<0, TN>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                const v4f &v = acc[t][j];
                if constexpr (ALONG_J) {
                    *reinterpret_cast<float4 *>(reg + lr * STRIDE + (j * 16 + 4 * lg) * 4) =
                        make_float4(v[0] * rd[t][0], v[1] * rd[t][0], v[2] * rd[t][0], v[3] * rd[t][0]);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<float *>(reg + (4 * lg + q) * STRIDE + (j * 16 + lr) * 4) = v[q] * rd[t][q];
                }
            });
        } else {
            static_for<0, TM>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                const v4f &v = acc[i][t];
                if constexpr (!ALONG_J) {
                    // four consecutive i of one j: four consecutive output columns
                    *reinterpret_cast<float4 *>(reg + lr * STRIDE + (i * 16 + 4 * lg) * 4) =
                        make_float4(v[0] * rd[t][0], v[1] * rd[t][0], v[2] * rd[t][0], v[3] * rd[t][0]);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        *reinterpret_cast<float *>(reg + (4 * lg + q) * STRIDE + (i * 16 + lr) * 4) = v[q] * rd[t][q];
                }
            });
        }
        wave_sync();
        // store 16-byte chunks of whole output rows, times the column descale
        for (int r = rsub; r < 16; r += rstep) {
            const int orow = orow0 + t * 16 + r;
            if (orow >= rows_out) break;
            const float *src = reinterpret_cast<const float *>(reg + r * STRIDE + cc * per * 4);
            float v[8];
            const float4 x0 = *reinterpret_cast<const float4 *>(src);
            v[0] = x0.x * cd[0]; v[1] = x0.y * cd[1]; v[2] = x0.z * cd[2]; v[3] = x0.w * cd[3];
            uint8_t *dst = reinterpret_cast<uint8_t *>(p.c) + ((int64_t)orow * p.ldc + ocol) * esz;
            const bool full = vec_ok && ocol + per <= cols_out;
            if (bf) {
                const float4 x1 = *reinterpret_cast<const float4 *>(src + 4);
                v[4] = x1.x * cd[4]; v[5] = x1.y * cd[5]; v[6] = x1.z * cd[6]; v[7] = x1.w * cd[7];
                uint16_t h[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) h[e] = f16 ? f32_to_f16_rne(v[e]) : f32_to_bf16_rne(v[e]);
                if (full) {
                    *reinterpret_cast<uint4 *>(dst) = make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16,
                                                                 h[4] | (uint32_t)h[5] << 16, h[6] | (uint32_t)h[7] << 16);
                } else {
                    for (int e = 0; e < 8 && ocol + e < cols_out; ++e) reinterpret_cast<uint16_t *>(dst)[e] = h[e];
                }
            } else {
                if (full) *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                else
                    for (int e = 0; e < 4 && ocol + e < cols_out; ++e) reinterpret_cast<float *>(dst)[e] = v[e];
            }
        }
        wave_sync();   // the next pass rewrites the region these reads use
    });
}

// Epilogue of a workgroup tile: every wave writes its accumulators to C.
// The output is staged through the wave's own region of LDS, sixteen output
// rows at a time, so that global stores are 16-byte chunks of whole rows
// (a wave writes 64 to 512 contiguous bytes of each row) instead of the
// 8-byte pieces of sixteen rows that one MFMA result holds.  Only the first
// pass waits for the whole workgroup (the main loop's LDS is shared); the
// passes themselves touch only the wave's own region.  The value is
// (acc * d_i) * d_j (transposed output: (acc * d_j) * d_i) in FP32: the
// staged value carries the output row's descale, the column's is applied
// when the row chunk is stored, as FP32, BF16 or FP16 (both RNE).  Split-K partial
// sums go to the workspace through store4 instead.  Every wave of the
// workgroup must call it (it synchronises the workgroup) once the main loop
// no longer touches LDS.  LDS_BYTES: LDS the tile owns.
template <int BM, int BN, int WM, int WN, bool ALONG_J, int LDS_BYTES>
__device__ __forceinline__ void write_tile(const GemmParams &p, const v4f (&acc)[BM / WM / 16][BN / WN / 16], int m0,
                                           int n0, int wave, int lane, int split, uint8_t *smem)
{
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lg = lane >> 4;
    if (p.splits > 1) {
        static_for<0, TM>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            static_for<0, TN>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                const int ib = m0 + wm * WTM + i * 16 + (ALONG_J ? lr : 4 * lg);
                const int jb = n0 + wn * WTN + j * 16 + (ALONG_J ? 4 * lg : lr);
                store4<ALONG_J>(p, ib, jb, split, acc[i][j]);
            });
        });
        return;
    }
    if (p.trans_out) write_tile_staged<BM, BN, WM, WN, ALONG_J, LDS_BYTES, true>(p, acc, m0, n0, wave, lane, smem);
    else write_tile_staged<BM, BN, WM, WN, ALONG_J, LDS_BYTES, false>(p, acc, m0, n0, wave, lane, smem);
}

// One 16-byte load per lane from a buffer resource straight into LDS: lane l
// writes LDS bytes [lds + 16 l, lds + 16 l + 16).  Issued from inline
// assembly so that the compiler does not treat the pending LDS write as a
// possible alias of every later LDS read (which would make it wait for the
// load before the fragment reads of the current stage); the caller waits for
// these loads with wait_vm before the barrier that publishes the stage.
// The instruction writes no register.  M0 carries the LDS address (bound as
// an input, so the compiler writes it).  The scalar operands are wave-uniform
// by construction; readfirstlane says so where the analysis cannot see it,
// which may leave a VALU write of the scalar offset right before the load.
// The compiler's hazard checks do not look inside the asm, so it waits the
// five states a vector memory read of a VALU-written SGPR needs (which also
// covers the one state after an M0 write).
__device__ __forceinline__ void dma16(uint32_t lds, int voff, __amdgpu_buffer_rsrc_t rs, int soff)
{
    const uint32_t m = __builtin_amdgcn_readfirstlane(lds);
    const int so = __builtin_amdgcn_readfirstlane(soff);
    asm volatile("s_nop 4\n\tbuffer_load_dwordx4 %0, %1, %2 offen lds"
                 :
                 : "v"(voff), "s"(rs), "s"(so), "{m0}"(m)
                 : "memory");
}

// A buffer resource whose pieces are wave-uniform by construction (the tile
// base and its byte range); readfirstlane makes that explicit, so the
// resource lives in scalar registers as the DMA instruction requires.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const uint8_t *base, int records)
{
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    void *u = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, __builtin_amdgcn_readfirstlane(records), kBufferFlags);
}

// s_waitcnt vmcnt(N) with the other counters left alone (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// FP8 -> BF16 with the hardware conversion, which is exact for every E4M3
// and E5M2 code (both fit BF16's exponent range and mantissa).
template <int FMT, bool HI>
__device__ __forceinline__ uint32_t fp8x2_to_bf16x2(uint32_t w)
{
    typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
    v2bf r;
    if constexpr (FMT == kE4M3) r = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)w, 1.0f, HI);
    else r = __builtin_amdgcn_cvt_scalef32_pk_bf16_bf8((int)w, 1.0f, HI);
    uint32_t u;
    __builtin_memcpy(&u, &r, 4);
    return u;
}

// 16 FP8 codes (little-endian in q) -> 16 BF16 as two 16-byte chunks
template <int FMT>
__device__ __forceinline__ void decode16(const uint4 &q, uint4 &lo, uint4 &hi)
{
    lo = make_uint4(fp8x2_to_bf16x2<FMT, false>(q.x), fp8x2_to_bf16x2<FMT, true>(q.x),
                    fp8x2_to_bf16x2<FMT, false>(q.y), fp8x2_to_bf16x2<FMT, true>(q.y));
    hi = make_uint4(fp8x2_to_bf16x2<FMT, false>(q.z), fp8x2_to_bf16x2<FMT, true>(q.z),
                    fp8x2_to_bf16x2<FMT, false>(q.w), fp8x2_to_bf16x2<FMT, true>(q.w));
}

// 16 kept codes of 32 dense positions (two per group of four, ascending) and
// their eight index nibbles -> the 32 dense codes (zeros elsewhere)
__device__ __forceinline__ void expand24(const uint4 &v, uint32_t meta, uint4 &d0, uint4 &d1)
{
    uint32_t kept[4] = {v.x, v.y, v.z, v.w}, dense[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        const uint32_t nib = (meta >> (4 * g)) & 15u;
        const uint32_t i0 = nib & 3u, i1 = nib >> 2;
        const uint32_t c0 = (kept[g / 2] >> (16 * (g & 1))) & 0xFFu, c1 = (kept[g / 2] >> (16 * (g & 1) + 8)) & 0xFFu;
        // group g occupies dense word g: byte i0 <- c0, byte i1 <- c1 (i0 < i1)
        dense[g] = (c0 << (8 * i0)) | (c1 << (8 * i1));
    }
    d0 = make_uint4(dense[0], dense[1], dense[2], dense[3]);
    d1 = make_uint4(dense[4], dense[5], dense[6], dense[7]);
}

// 8 kept codes of 16 dense positions (two per group of four, ascending) and
// their four index nibbles -> the 16 dense codes (zeros elsewhere)
__device__ __forceinline__ uint4 expand24_half(uint2 v, uint32_t nibs)
{
    uint32_t d[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const uint32_t nib = (nibs >> (4 * g)) & 15u;
        const uint32_t kw = g < 2 ? v.x : v.y, sh = 16 * (g & 1);
        const uint32_t c0 = (kw >> sh) & 0xFFu, c1 = (kw >> (sh + 8)) & 0xFFu;
        d[g] = (c0 << (8 * (nib & 3u))) | (c1 << (8 * (nib >> 2)));
    }
    return make_uint4(d[0], d[1], d[2], d[3]);
}

// LDS-DMA pipeline (PF >= 6: NS = PF - 4 LDS stages).  Global tiles go
// straight from memory into LDS without passing through registers, which
// frees the staging registers for larger wave tiles (a 128 x 128 wave tile
// reads half the LDS bytes per MFMA of a 64 x 64 one).  Each 1 KiB block of
// a stage is filled by one wave instruction; the lane that writes slot c' of
// row r fetches global chunk c' ^ swizzle(r), so LDS holds the same swizzled
// layout the fragment reads expect.  Chunks past the end of K are fetched
// from an offset beyond the resource range, which the hardware returns as
// zero.  Step k: wait for stage k (own loads), barrier (everyone's loads;
// everyone done reading stage k - 1), issue stage k + NS - 1 into the buffer
// of step k - 1, MFMAs of stage k.  One stage is issued per step whatever k
// is (past the last step into a buffer nobody reads), so the wait count is a
// constant; everything is drained before the workgroup ends.  Requires K to
// be a multiple of 16 (dense) or 128 (compressed operand).
// HP >= 0: the operands are FP32, FP16 or BF16 values instead of FP8 codes
// (kHpF32 / kHpF16 / kHpBF16); p.K, p.kchunk, p.lda and p.ldb then count
// bytes, so a step covers 128 bytes of K (32 or 64 elements), and each lane
// reads chunk 4 h + g of its rows (h = 0, 1): 8 elements for one 16-bit MFMA,
// 4 for four FP32 ones (instruction t takes element t), the same k mapping in
// A and B.
template <int BM, int BN, int WM, int WN, int FA, int FB, bool SP, int NS, int PF, bool SWAP, int HP = -1>
__device__ __forceinline__ void gemm_tile_dma(const GemmParams &p, int tm, int tn, int split, uint8_t *smem)
{
    constexpr int NW = WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    using S = TileSmem<BM, BN, SP, PF>;
    static_assert(S::NSTAGE == NS, "stage count");
    constexpr int QA = S::A_BYTES / 1024, QM = S::M_BYTES / 1024, QB = S::B_BYTES / 1024;
    static_assert(S::A_BYTES % 1024 == 0 && S::M_BYTES % 1024 == 0 && S::B_BYTES % 1024 == 0, "1 KiB blocks");
    // Loader waves.  With two waves per SIMD (NW = 8), only waves 0-3 (one
    // per SIMD) issue the loads: a wave waits at each load until the texture
    // path takes it, and a CU's loads of a stage take that path about 1000
    // cycles, so if both waves of a SIMD issued loads after the barrier both
    // would wait and the matrix core would idle; this way the other wave of
    // each SIMD runs its MFMAs meanwhile.
    constexpr int ND = (NW == 8 && QA % 4 == 0 && QB % 4 == 0 && (QM % 4 == 0 || QM < 4)) ? 4 : NW;
    static_assert(QM % ND == 0 || QM < ND, "metadata blocks per wave");
    // full rounds per loader wave per stage; the first QA % ND (QB % ND)
    // loader waves take one more A (B) block
    constexpr int RA = QA / ND, RB = QB / ND, RM = QM / ND;
    constexpr int XA = QA % ND, XB = QB % ND;
    constexpr int PER = RA + RB + RM;                          // DMA instructions per loader wave per stage (at least)
    static_assert((NS - 2) * PER < 64, "vmcnt range");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lg = lane >> 4;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kbeg = split * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);
    const int nk = (kend - kbeg + kBK - 1) / kBK;
    const int Kv = p.K / 2, Km = p.K / 8;

    const int rows_a = min(BM, p.M - m0), rows_b = min(BN, p.N - n0);
    const int rec_a = rows_a * (int)p.lda, rec_b = rows_b * (int)p.ldb, rec_m = SP ? rows_a * (int)p.ldm : 0;
    const __amdgpu_buffer_rsrc_t rs_a = uniform_rsrc(p.a + (int64_t)m0 * p.lda, rec_a);
    const __amdgpu_buffer_rsrc_t rs_b = uniform_rsrc(p.b + (int64_t)n0 * p.ldb, rec_b);
    const __amdgpu_buffer_rsrc_t rs_m = uniform_rsrc(SP ? p.meta + (int64_t)m0 * p.ldm : p.a, rec_m);

    // Per-lane source of the first block a loader wave fills; later rounds
    // move down by ND blocks (a whole number of rows).  Dense rows (128 bytes):
    // block q holds rows 8q .. 8q+7, lane l row 8q + l/8, slot l%8, so the
    // source chunk is (l%8) ^ (l/8) ^ (q&1); round u of an odd number of
    // waves flips the last term, so a second offset serves those rounds.
    const int cd = (lane & 7) ^ (lane >> 3) ^ (wave & 1);
    // B rows of a 2:4 kernel use swz_b2: the block-parity term flips bit 1
    const int fb = SP ? 2 : 1;
    const int cb = (lane & 7) ^ (lane >> 3) ^ ((wave & 1) ? fb : 0);
    const int voff_b = (wave * 8 + (lane >> 3)) * (int)p.ldb + cb * 16;
    // A: dense as B; compressed values (64 bytes): block q holds rows 16q ..
    // 16q+15, lane l row 16q + l/4, slot l%4, chunk
    // (l%4) ^ ((l>>3)&1) ^ ((l>>5) << 1) (swz_sp).
    const int cs = (lane & 3) ^ ((lane >> 3) & 1) ^ ((lane >> 5) << 1);
    const int ca = SP ? cs : cd;
    const int voff_a = SP ? (wave * 16 + (lane >> 2)) * (int)p.lda + cs * 16 : (wave * 8 + (lane >> 3)) * (int)p.lda + cd * 16;
    // metadata (16 bytes per row): block q holds rows 64q .. 64q+63.
    const int voff_m = (wave * 64 + lane) * (int)p.ldm;
    const uint32_t lds0 = (uint32_t)(uintptr_t)smem;

    const bool loader = wave < ND;
    auto issue = [&](int kt, int stage) {
        if (!loader) return;
        const int k0 = kbeg + kt * kBK;
        const uint32_t sb = lds0 + stage * S::STAGE;
        // whole chunks past the end of K read as zero: point them past the range
        const int va = SP ? (k0 / 2 + ca * 16 < Kv ? voff_a : rec_a) : (k0 + ca * 16 < kend ? voff_a : rec_a);
        const int vb = k0 + cb * 16 < kend ? voff_b : rec_b;
        // rounds whose block parity differs from the first one's (odd NW)
        const int cdf = cd ^ 1, cbf = cb ^ fb;
        const int vaf = SP ? va : (k0 + cdf * 16 < kend ? voff_a + (cdf - cd) * 16 : rec_a);
        const int vbf = k0 + cbf * 16 < kend ? voff_b + (cbf - cb) * 16 : rec_b;
        constexpr int rows_a_blk = SP ? 16 : 8;   // rows per 1 KiB block
        static_for<0, RA>([&](auto uu) {
            constexpr int u = decltype(uu)::value;
            dma16(sb + (wave + u * ND) * 1024, ((u * ND) & 1) ? vaf : va, rs_a,
                  u * ND * rows_a_blk * (int)p.lda + (SP ? k0 / 2 : k0));
        });
        if constexpr (XA > 0) {
            if (wave < XA)
                dma16(sb + (wave + RA * ND) * 1024, ((RA * ND) & 1) ? vaf : va, rs_a,
                      RA * ND * rows_a_blk * (int)p.lda + (SP ? k0 / 2 : k0));
        }
        if constexpr (SP) {
            const int vm = k0 / 8 < Km ? voff_m : rec_m;
            if constexpr (RM > 0) {
                static_for<0, RM>([&](auto uu) {
                    constexpr int u = decltype(uu)::value;
                    dma16(sb + S::A_BYTES + (wave + u * ND) * 1024, vm, rs_m, u * ND * 64 * (int)p.ldm + k0 / 8);
                });
            } else {
                if (wave < QM) dma16(sb + S::A_BYTES + wave * 1024, vm, rs_m, k0 / 8);
            }
        }
        static_for<0, RB>([&](auto uu) {
            constexpr int u = decltype(uu)::value;
            dma16(sb + S::A_BYTES + S::M_BYTES + (wave + u * ND) * 1024, ((u * ND) & 1) ? vbf : vb, rs_b,
                  u * ND * 8 * (int)p.ldb + k0);
        });
        if constexpr (XB > 0) {
            if (wave < XB)
                dma16(sb + S::A_BYTES + S::M_BYTES + (wave + RB * ND) * 1024, ((RB * ND) & 1) ? vbf : vb, rs_b,
                      RB * ND * 8 * (int)p.ldb + k0);
        }
    };

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    // Fragment addresses: rows 16 apart share their swizzle phase, so every
    // fragment of a wave is one per-lane base plus a compile-time offset
    // (2048 bytes per 16 dense rows, 1024 per 16 compressed rows, 256 per
    // 16 metadata rows).
    const int rb0 = wn * WTN + lr, ra0 = wm * WTM + lr;
    const int ob0 = S::A_BYTES + S::M_BYTES + swz_b<SP>(rb0, SP ? lg : 2 * lg);
    const int ob1 = S::A_BYTES + S::M_BYTES + swz_b<SP>(rb0, SP ? lg + 4 : 2 * lg + 1);
    const int oa0 = SP ? swz_sp(ra0, lg) : swz(ra0, 2 * lg);
    const int oa1 = SP ? S::A_BYTES + ra0 * 16 + lg * 4 : swz(ra0, 2 * lg + 1);
    // Exact sums (pf_exact_dma): each lane reads 16-byte chunk 4 h + lg of
    // its rows (h = 0, 1; conflict-free under swz, as every lane of a 16-row
    // group reads the same chunk) and decodes it to 16 BF16; lane group lg
    // feeds codes 64 h + 16 lg .. + 7 to one BF16 MFMA (32 k each) and the
    // next eight to a second, in both operands, so the four MFMAs of a step
    // cover its 128 k once each.
    typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
    auto as_bf = [](const uint4 &v) {
        v8bf f;
        __builtin_memcpy(&f, &v, 16);
        return f;
    };
    auto compute_exact = [&](int stage) {
        const uint8_t *base = smem + stage * S::STAGE;
        static_for<0, 2>([&](auto hh) {
            constexpr int h = decltype(hh)::value;
            const int ob = S::A_BYTES + swz(rb0, 4 * h + lg), oa = swz(ra0, 4 * h + lg);
            v8bf blo[TN], bhi[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                uint4 lo, hi;
                decode16<FB>(*reinterpret_cast<const uint4 *>(base + ob + j * 2048), lo, hi);
                blo[j] = as_bf(lo);
                bhi[j] = as_bf(hi);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                uint4 lo, hi;
                decode16<FA>(*reinterpret_cast<const uint4 *>(base + oa + i * 2048), lo, hi);
                const v8bf alo = as_bf(lo), ahi = as_bf(hi);
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if constexpr (SWAP) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(blo[j], alo, acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bhi[j], ahi, acc[i][j], 0, 0, 0);
                    } else {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, blo[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi[j], acc[i][j], 0, 0, 0);
                    }
                }
            }
        });
    };
    // The same with a compressed A.  Here lane group g feeds dense chunk
    // 2 g + h in pass h (A and B alike): one 128-bit read of compressed
    // chunk g (16 kept codes) and its 32-bit index word cover both passes,
    // the same reads the 2:4 FP8 instruction makes; the 32 dense codes they
    // expand to are decoded once per step.
    auto compute_exact_sp = [&](int stage) {
        const uint8_t *base = smem + stage * S::STAGE;
        v8bf blo[2][TN], bhi[2][TN];
        static_for<0, 2>([&](auto hh) {
            constexpr int h = decltype(hh)::value;
            const int ob = S::A_BYTES + S::M_BYTES + swz_b2(rb0, 2 * lg + h);
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                uint4 lo, hi;
                decode16<FB>(*reinterpret_cast<const uint4 *>(base + ob + j * 2048), lo, hi);
                blo[h][j] = as_bf(lo);
                bhi[h][j] = as_bf(hi);
            }
        });
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const uint4 kept = *reinterpret_cast<const uint4 *>(base + oa0 + i * 1024);
            const uint32_t meta = *reinterpret_cast<const uint32_t *>(base + oa1 + i * 256);
            uint4 d0, d1, l0, h0, l1, h1;
            expand24(kept, meta, d0, d1);
            decode16<FA>(d0, l0, h0);
            decode16<FA>(d1, l1, h1);
            const v8bf a[4] = {as_bf(l0), as_bf(h0), as_bf(l1), as_bf(h1)};
            // (the four MFMAs into one accumulator are TN instructions apart)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        a[t], (t & 1) ? bhi[t >> 1][j] : blo[t >> 1][j], acc[i][j], 0, 0, 0);
        }
    };
    auto compute_hp = [&](int stage) {
        static_assert(HP < 0 || (!SP && !pf_exact_dma(PF)), "higher-precision operands: dense FP8-layout ring");
        const uint8_t *base = smem + stage * S::STAGE;
        static_for<0, 2>([&](auto hh) {
            constexpr int h = decltype(hh)::value;
            const int ob = S::A_BYTES + swz(rb0, 4 * h + lg), oa = swz(ra0, 4 * h + lg);
            uint4 bq[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) bq[j] = *reinterpret_cast<const uint4 *>(base + ob + j * 2048);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const uint4 aq = *reinterpret_cast<const uint4 *>(base + oa + i * 2048);
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    // SWAP: B rows in the instruction's A slot (row-major output lanes)
                    const uint4 &x = SWAP ? bq[j] : aq, &y = SWAP ? aq : bq[j];
                    if constexpr (HP == kHpF32) {
                        const uint32_t x4[4] = {x.x, x.y, x.z, x.w}, y4[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(x4[t]),
                                                                             __uint_as_float(y4[t]), acc[i][j], 0, 0, 0);
                    } else if constexpr (HP == kHpF16) {
                        typedef _Float16 v8h __attribute__((ext_vector_type(8)));
                        v8h x8, y8;
                        __builtin_memcpy(&x8, &x, 16);
                        __builtin_memcpy(&y8, &y, 16);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x8, y8, acc[i][j], 0, 0, 0);
                    } else {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(x), as_bf(y), acc[i][j], 0, 0, 0);
                    }
                }
            }
        });
    };
    // 32 x 32 x 64 instructions (pf_mfma32): lane l supplies row l % 32 and
    // codes 32 g .. 32 g + 31 (g = l / 32) of each 64-code half hk of the
    // step, i.e. chunks 4 hk + 2 g and 4 hk + 2 g + 1; rows 32 apart share
    // their swizzle phase.  Each 32 x 32 block accumulates in 16 registers.
    constexpr int TM2 = TM / 2 > 0 ? TM / 2 : 1, TN2 = TN / 2 > 0 ? TN / 2 : 1;
    v16f acc32[TM2][TN2];
    if constexpr (pf_mfma32(PF)) {
        static_assert(TM % 2 == 0 && TN % 2 == 0 && !SP && !SWAP, "32 x 32 blocks");
#pragma unroll
        for (int i = 0; i < TM2; ++i)
#pragma unroll
            for (int j = 0; j < TN2; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc32[i][j][e] = 0.f;
    }
    const int r32 = lane & 31, g32 = lane >> 5;
    const int ra32 = wm * WTM + r32, rb32 = wn * WTN + r32;
    auto compute_32 = [&](int stage) {
        const uint8_t *base = smem + stage * S::STAGE;
        static_for<0, 2>([&](auto hh) {
            constexpr int hk = decltype(hh)::value;
            const int c0 = 4 * hk + 2 * g32;
            const int ob = S::A_BYTES + swz(rb32, c0), ob1 = S::A_BYTES + swz(rb32, c0 + 1);
            const int oa = swz(ra32, c0), oa1 = swz(ra32, c0 + 1);
            v8i bf[TN2];
#pragma unroll
            for (int j = 0; j < TN2; ++j) {
                const uint4 lo = *reinterpret_cast<const uint4 *>(base + ob + j * 4096);
                const uint4 hi = *reinterpret_cast<const uint4 *>(base + ob1 + j * 4096);
                bf[j] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
#pragma unroll
            for (int i = 0; i < TM2; ++i) {
                const uint4 lo = *reinterpret_cast<const uint4 *>(base + oa + i * 4096);
                const uint4 hi = *reinterpret_cast<const uint4 *>(base + oa1 + i * 4096);
                const v8i af = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
#pragma unroll
                for (int j = 0; j < TN2; ++j)
                    acc32[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af, bf[j], acc32[i][j], FA, FB, 0, 0,
                                                                                 0, 0);
            }
        });
    };
    auto compute = [&](int stage) {
        if constexpr (pf_mfma32(PF)) {
            compute_32(stage);
            return;
        }
        if constexpr (HP >= 0) {
            compute_hp(stage);
            return;
        }
        if constexpr (pf_exact_dma(PF)) {
            if constexpr (SP) compute_exact_sp(stage);
            else compute_exact(stage);
            return;
        }
        const uint8_t *base = smem + stage * S::STAGE;
        v8i bf[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            uint4 lo = *reinterpret_cast<const uint4 *>(base + ob0 + j * 2048);
            uint4 hi = *reinterpret_cast<const uint4 *>(base + ob1 + j * 2048);
            bf[j] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            if constexpr (SP) {
                uint4 v = *reinterpret_cast<const uint4 *>(base + oa0 + i * 1024);
                const int idx = *reinterpret_cast<const int *>(base + oa1 + i * 256);
                v4i af = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma_sparse<FA, FB>(af, bf[j], acc[i][j], idx);
            } else {
                uint4 lo = *reinterpret_cast<const uint4 *>(base + oa0 + i * 2048);
                uint4 hi = *reinterpret_cast<const uint4 *>(base + oa1 + i * 2048);
                v8i af = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if constexpr (SWAP) acc[i][j] = mfma_dense<FB, FA>(bf[j], af, acc[i][j]);
                    else acc[i][j] = mfma_dense<FA, FB>(af, bf[j], acc[i][j]);
                }
            }
        }
    };

    if (nk > 0) {
        static_for<0, NS - 1>([&](auto ss) {
            constexpr int s = decltype(ss)::value;
            issue(s, s);
        });
        int st = 0, nx = NS - 1;   // stage of step kt, stage of step kt + NS - 1
        for (int kt = 0; kt < nk; ++kt) {
            wait_vm<(NS - 2) * PER>();
            __syncthreads();
            issue(kt + NS - 1, nx);
            compute(st);
            st = st + 1 == NS ? 0 : st + 1;
            nx = nx + 1 == NS ? 0 : nx + 1;
        }
        wait_vm<0>();
    }

    if constexpr (pf_mfma32(PF)) {
        // Each 32 x 32 block to the four 16 x 16 blocks the epilogue takes.
        // 32 x 32 layout: element (i, j) in lane j + 32 ((i / 4) % 2),
        // register (i % 4) + 4 (i / 8).  16 x 16 layout (unswapped): lane L
        // holds rows 4 (L / 16) .. + 3 of column L % 16.  So value q of lane L
        // in 16 x 16 block (a, b) comes from lane 16 b + L % 16 + 32 ((L / 16)
        // % 2), register 8 a + 4 (L / 32) + q.
        static_for<0, TM2>([&](auto ii) {
            constexpr int i2 = decltype(ii)::value;
            static_for<0, TN2>([&](auto jj) {
                constexpr int j2 = decltype(jj)::value;
                const v16f x = acc32[i2][j2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int src = (16 * b + (lane & 15) + 32 * ((lane >> 4) & 1)) * 4;
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int y0 = __builtin_amdgcn_ds_bpermute(src, __float_as_int(x[8 * a + q]));
                            const int y1 = __builtin_amdgcn_ds_bpermute(src, __float_as_int(x[8 * a + 4 + q]));
                            acc[2 * i2 + a][2 * j2 + b][q] = __int_as_float(lane < 32 ? y0 : y1);
                        }
                    }
                }
            });
        });
    }
    static_assert(!(SP && SWAP), "the compressed operand must stay in the MFMA A slot");
    write_tile<BM, BN, WM, WN, SWAP, S::TOTAL>(p, acc, m0, n0, wave, lane, split, smem);
}

// Exact-sum pipeline (PF == kExactPF).  gfx950's FP8 MFMAs add each run of
// eight consecutive-k products after aligning them to the largest exponent
// sum of the run and keep only about fourteen bits below it, so their error
// is bounded by about 2^-13 of the largest product of each run: inside
// 4 K 2^-24 sum |a b| for every input only once K >= 3584.  This pipeline
// decodes the FP8 codes exactly to BF16 (the hardware conversion is exact
// for every E4M3 and E5M2 code) and multiplies on the BF16 MFMA
// (v_mfma_f32_16x16x32_bf16), whose products are exact and whose sums keep
// 23 bits below the largest product of an instruction, so the bound holds
// for every K.  Loads go through registers: the codes of step k + 3 are
// loaded at the start of step k (three register sets), and those of step
// k + 1 are decoded into the other of two LDS stages between the MFMAs of
// step k.  A 2:4 operand (values + index nibbles) is expanded to its dense
// row while it is decoded, after which the step is a dense one.  LDS rows
// hold 128 BF16 (256 bytes) with 16-byte chunk x of row r at x ^ (r & 15);
// lane l reads row l % 16, codes 8 (l / 16) .. 8 (l / 16) + 7 of each 32
// (one chunk), for both operands; a lane's result is four consecutive i of
// one j.  (Dense operands with K a multiple of 16 also have the exact-sum DMA
// ring, pf_exact_dma, which keeps FP8 codes in LDS and decodes after the
// fragment reads: half the LDS bytes per step.)


// Codes [k, k + 16) of a row of `len` codes, zero past the end (byte-exact
// when the chunk is partial or unaligned).
__device__ __forceinline__ uint4 load_codes16(const uint8_t *row, int k, int len)
{
    if (k + 16 <= len && ((reinterpret_cast<uintptr_t>(row + k) & 15) == 0))
        return *reinterpret_cast<const uint4 *>(row + k);
    return load16_partial(row + k, max(0, min(16, len - k)), 0u);
}

template <int BM, int BN, int WM, int WN, int FA, int FB, bool SP, bool SPB = false, bool KFAST = true>
__device__ __forceinline__ void gemm_tile_exact(const GemmParams &p, int tm, int tn, int split, uint8_t *smem)
{
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    using S = TileSmem<BM, BN, SP, kExactPF>;
    // work units per step: dense rows have 8 chunks of 16 codes, compressed
    // rows 4 chunks of 16 kept codes (32 dense positions each)
    constexpr int A_U = SP ? BM * 4 : BM * 8, B_U = SPB ? BN * 4 : BN * 8;
    constexpr int A_PER = (A_U + NT - 1) / NT, B_PER = (B_U + NT - 1) / NT;
    static_assert(TM >= 1 && TN >= 1, "wave tile");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lg = lane >> 4;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kbeg = split * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);
    const int nk = (kend - kbeg + kBK - 1) / kBK;
    const int Kv = p.K / 2, Km = p.K / 8;

    // NSET register sets: the loads of step k + NSET are issued at the start
    // of step k, so global latency is hidden behind NSET steps of MFMAs
    constexpr int NSET = 3;
    uint4 ra[NSET][A_PER], rb[NSET][B_PER];
    uint32_t rm[NSET][SP ? A_PER : 1], rmb[NSET][SPB ? B_PER : 1];
    // Fast path (K a multiple of 16, or of 128 for a compressed operand):
    // every chunk is one unconditional buffer load against a per-tile
    // resource whose range ends at the last valid row, so rows past M or N
    // read as zero, and a chunk past the end of the K range is pointed at the
    // end of the range and reads as zero too.  With no branches around the
    // loads the compiler counts them exactly and waits only for the set a
    // store uses, not for every load in flight.
    static_assert(NT % 8 == 0, "a thread keeps its chunk column across units");
    const int rows_a = min(BM, p.M - m0), rows_b = min(BN, p.N - n0);
    const int rec_a = rows_a * (int)p.lda, rec_b = rows_b * (int)p.ldb;
    const int rec_m = SP ? rows_a * (int)p.ldm : 0, rec_mb = SPB ? rows_b * (int)p.ldmb : 0;
    const __amdgpu_buffer_rsrc_t rs_a = uniform_rsrc(p.a + (int64_t)m0 * p.lda, rec_a);
    const __amdgpu_buffer_rsrc_t rs_b = uniform_rsrc(p.b + (int64_t)n0 * p.ldb, rec_b);
    const __amdgpu_buffer_rsrc_t rs_m = uniform_rsrc(SP ? p.meta + (int64_t)m0 * p.ldm : p.a, rec_m);
    const __amdgpu_buffer_rsrc_t rs_mb = uniform_rsrc(SPB ? p.meta_b + (int64_t)n0 * p.ldmb : p.b, rec_mb);
    // dense rows: unit u of a thread is row tid / 8 + u NT / 8, chunk tid % 8;
    // compressed rows: row tid / 4 + u NT / 4, chunk tid % 4 (32 dense codes)
    const int ca = SP ? (tid & 3) : (tid & 7), cb = SPB ? (tid & 3) : (tid & 7);
    const int voff_a = SP ? (tid >> 2) * (int)p.lda + ca * 16 : (tid >> 3) * (int)p.lda + ca * 16;
    const int voff_b = SPB ? (tid >> 2) * (int)p.ldb + cb * 16 : (tid >> 3) * (int)p.ldb + cb * 16;
    const int voff_m = (tid >> 2) * (int)p.ldm + ca * 4, voff_mb = (tid >> 2) * (int)p.ldmb + cb * 4;
    auto bload = [](const __amdgpu_buffer_rsrc_t &r, int voff, int soff) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        return make_uint4(v[0], v[1], v[2], v[3]);
    };
    auto gload_fast = [&](int kt, auto ss) {
        constexpr int st = decltype(ss)::value;
        const int k0 = kbeg + kt * kBK;
        // (the step's chunk column is the same for every unit of a thread)
        const bool va = SP ? k0 / 2 + ca * 16 < kend / 2 : k0 + ca * 16 < kend;
        const bool vb = SPB ? k0 / 2 + cb * 16 < kend / 2 : k0 + cb * 16 < kend;
        const bool vm = k0 / 8 + ca * 4 < kend / 8, vmb = k0 / 8 + cb * 4 < kend / 8;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            if (A_U % NT != 0 && tid + u * NT >= A_U) break;
            constexpr int RPU = SP ? NT / 4 : NT / 8;   // rows per unit
            ra[st][u] = bload(rs_a, va ? voff_a + u * RPU * (int)p.lda : rec_a, SP ? k0 / 2 : k0);
            if constexpr (SP)
                rm[st][u] = __builtin_amdgcn_raw_buffer_load_b32(rs_m, vm ? voff_m + u * RPU * (int)p.ldm : rec_m,
                                                                 k0 / 8, 0);
        }
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            if (B_U % NT != 0 && tid + u * NT >= B_U) break;
            constexpr int RPU = SPB ? NT / 4 : NT / 8;
            rb[st][u] = bload(rs_b, vb ? voff_b + u * RPU * (int)p.ldb : rec_b, SPB ? k0 / 2 : k0);
            if constexpr (SPB)
                rmb[st][u] = __builtin_amdgcn_raw_buffer_load_b32(
                    rs_mb, vmb ? voff_mb + u * RPU * (int)p.ldmb : rec_mb, k0 / 8, 0);
        }
    };
    // Byte-exact path (any K): rows and chunks are clipped one by one.
    auto gload = [&](int kt, auto ss) {
        if constexpr (KFAST) {
            gload_fast(kt, ss);
            return;
        }
        constexpr int st = decltype(ss)::value;
        const int k0 = kbeg + kt * kBK;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_U % NT != 0 && idx >= A_U) break;
            if constexpr (SP) {
                const int r = idx >> 2, c = idx & 3, row = m0 + r;
                // kept codes of dense positions [k0 + 32 c, k0 + 32 c + 32)
                const int vk = k0 / 2 + 16 * c;
                const int lim = min(Kv, kend / 2);
                ra[st][u] = row < p.M ? load_codes16(p.a + (int64_t)row * p.lda, vk, lim) : make_uint4(0, 0, 0, 0);
                uint32_t m = 0;
                if (row < p.M) {
                    const uint8_t *mr = p.meta + (int64_t)row * p.ldm + k0 / 8 + 4 * c;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (k0 / 8 + 4 * c + b < min(Km, kend / 8)) m |= (uint32_t)mr[b] << (8 * b);
                }
                rm[st][u] = m;
            } else {
                const int r = idx >> 3, c = idx & 7, row = m0 + r;
                ra[st][u] = row < p.M ? load_codes16(p.a + (int64_t)row * p.lda, k0 + 16 * c, kend) : make_uint4(0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_U % NT != 0 && idx >= B_U) break;
            if constexpr (SPB) {
                const int r = idx >> 2, c = idx & 3, row = n0 + r;
                const int vk = k0 / 2 + 16 * c;
                const int lim = min(Kv, kend / 2);
                rb[st][u] = row < p.N ? load_codes16(p.b + (int64_t)row * p.ldb, vk, lim) : make_uint4(0, 0, 0, 0);
                uint32_t m = 0;
                if (row < p.N) {
                    const uint8_t *mr = p.meta_b + (int64_t)row * p.ldmb + k0 / 8 + 4 * c;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (k0 / 8 + 4 * c + b < min(Km, kend / 8)) m |= (uint32_t)mr[b] << (8 * b);
                }
                rmb[st][u] = m;
            } else {
                const int r = idx >> 3, c = idx & 7, row = n0 + r;
                rb[st][u] = row < p.N ? load_codes16(p.b + (int64_t)row * p.ldb, k0 + 16 * c, kend) : make_uint4(0, 0, 0, 0);
            }
        }
    };
    // BF16 chunk x (8 codes) of row r sits at 16-byte slot x ^ (r & 15)
    auto put = [&](uint8_t *base, int r, int x, const uint4 &v) {
        *reinterpret_cast<uint4 *>(base + r * 256 + ((x ^ (r & 15)) << 4)) = v;
    };
    // One register unit into LDS stage `buf`: units 0 .. A_PER - 1 are the A
    // chunks of this thread, the next B_PER the B chunks.
    constexpr int QT = A_PER + B_PER;
    auto store_unit = [&](int buf, auto ss, auto qq) {
        constexpr int st = decltype(ss)::value, q = decltype(qq)::value;
        uint8_t *base = smem + buf * S::STAGE;
        if constexpr (q < A_PER) {
            constexpr int u = q;
            const int idx = tid + u * NT;
            if (A_U % NT != 0 && idx >= A_U) return;
            if constexpr (SP) {
                const int r = idx >> 2, c = idx & 3;
                uint4 d0, d1, b0, b1, b2, b3;
                expand24(ra[st][u], rm[st][u], d0, d1);
                decode16<FA>(d0, b0, b1);
                decode16<FA>(d1, b2, b3);
                put(base, r, 4 * c, b0);
                put(base, r, 4 * c + 1, b1);
                put(base, r, 4 * c + 2, b2);
                put(base, r, 4 * c + 3, b3);
            } else {
                const int r = idx >> 3, c = idx & 7;
                uint4 lo, hi;
                decode16<FA>(ra[st][u], lo, hi);
                put(base, r, 2 * c, lo);
                put(base, r, 2 * c + 1, hi);
            }
        } else {
            constexpr int u = q - A_PER;
            uint8_t *bb = base + S::A_BYTES;
            const int idx = tid + u * NT;
            if (B_U % NT != 0 && idx >= B_U) return;
            if constexpr (SPB) {
                const int r = idx >> 2, c = idx & 3;
                uint4 d0, d1, b0, b1, b2, b3;
                expand24(rb[st][u], rmb[st][u], d0, d1);
                decode16<FB>(d0, b0, b1);
                decode16<FB>(d1, b2, b3);
                put(bb, r, 4 * c, b0);
                put(bb, r, 4 * c + 1, b1);
                put(bb, r, 4 * c + 2, b2);
                put(bb, r, 4 * c + 3, b3);
            } else {
                const int r = idx >> 3, c = idx & 7;
                uint4 lo, hi;
                decode16<FB>(rb[st][u], lo, hi);
                put(bb, r, 2 * c, lo);
                put(bb, r, 2 * c + 1, hi);
            }
        }
    };
    auto sstore = [&](int buf, auto ss) {
        static_for<0, QT>([&](auto qq) { store_unit(buf, ss, qq); });
    };

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
    auto frag = [&](const uint8_t *base, int r, int x) {
        const uint4 v = *reinterpret_cast<const uint4 *>(base + r * 256 + ((x ^ (r & 15)) << 4));
        v8bf f;
        __builtin_memcpy(&f, &v, 16);
        return f;
    };
    // MFMAs of the step in LDS stage `buf`, four sub-steps of 32 codes; when
    // `store` is set, the decode and LDS stores of the next step's register
    // set (stage nbuf) follow each sub-step's MFMAs a quarter at a time, so
    // they run while the matrix core works instead of after it.
    auto compute = [&](int buf, int nbuf, bool store, auto ns) {
        const uint8_t *base = smem + buf * S::STAGE;
        const uint8_t *bb = base + S::A_BYTES;
        static_for<0, 4>([&](auto cc) {   // 32 codes of K per instruction
            constexpr int c = decltype(cc)::value;
            v8bf bf[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = frag(bb, wn * WTN + j * 16 + lr, 4 * c + lg);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const v8bf af = frag(base, wm * WTM + i * 16 + lr, 4 * c + lg);
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j], acc[i][j], 0, 0, 0);
            }
            if (store) static_for<c * QT / 4, (c + 1) * QT / 4>([&](auto qq) { store_unit(nbuf, ns, qq); });
        });
    };

    if (nk > 0) {
        static_for<0, NSET>([&](auto ss) {
            if (decltype(ss)::value < nk) gload(decltype(ss)::value, ss);
        });
        sstore(0, std::integral_constant<int, 0>{});
        __syncthreads();
        // step k: loads of step k + NSET into the set step k used; MFMAs on
        // LDS stage k % 2; step k + 1's set into the other stage; barrier
        for (int kt0 = 0; kt0 < nk; kt0 += NSET) {
            static_for<0, NSET>([&](auto ss) {
                constexpr int st = decltype(ss)::value;
                const int kt = kt0 + st;
                if (kt < nk) {
                    if (kt + NSET < nk) gload(kt + NSET, ss);
                    compute(kt & 1, (kt + 1) & 1, kt + 1 < nk, std::integral_constant<int, (st + 1) % NSET>{});
                    __syncthreads();
                }
            });
        }
    }
    write_tile<BM, BN, WM, WN, false, S::TOTAL>(p, acc, m0, n0, wave, lane, split, smem);
}

// Computes tile (tm, tn) of split `split`.  smem: TileSmem<BM,BN,SP>::TOTAL bytes.
// KFAST: K is a multiple of 16 (dense) or 128 (compressed operand), so every
// 16-byte chunk is either wholly inside the operand or wholly outside.
// PF: pipeline.  2: two register sets, global loads two steps ahead; 1: one
// step ahead; 3: three LDS stages and fragments read one step ahead; 6 and
// up: global -> LDS DMA with PF - 4 LDS stages (gemm_tile_dma).
// SWAP (dense only): run the MFMA with B rows in its A slot, so a lane ends
// up with four consecutive j of one i (vector stores for a row-major output);
// without it a lane holds four consecutive i of one j, which suits a
// transposed output.  The 2:4 path never swaps (the compressed operand must
// sit in the A slot).
template <int BM, int BN, int WM, int WN, int FA, int FB, bool SP, bool KFAST = true, int PF = 2,
          bool SWAP = !SP, bool SPB = false>
__device__ __forceinline__ void gemm_tile(const GemmParams &p, int tm, int tn, int split, uint8_t *smem)
{
    if constexpr (PF == kExactPF) {
        gemm_tile_exact<BM, BN, WM, WN, FA, FB, SP, SPB, KFAST>(p, tm, tn, split, smem);
        return;
    } else if constexpr (pf_mfma32(PF)) {
        static_assert(KFAST && !SP && !SPB, "32 x 32 MFMA ring: dense operands, whole 16-byte chunks");
        gemm_tile_dma<BM, BN, WM, WN, FA, FB, false, PF - 54, PF, false>(p, tm, tn, split, smem);
        return;
    } else if constexpr (pf_exact_dma(PF)) {
        static_assert(KFAST && !SPB, "exact sums on the DMA ring: whole 16-byte chunks, dense j operand");
        gemm_tile_dma<BM, BN, WM, WN, FA, FB, SP, PF - kExactPF, PF, SWAP>(p, tm, tn, split, smem);
        return;
    } else if constexpr (PF >= 6) {
        static_assert(KFAST, "the DMA pipeline needs whole 16-byte chunks");
        static_assert(!SPB, "a compressed j operand takes the register pipeline");
        if constexpr (SP && BM % 64 != 0) {
            // the metadata of fewer than 64 rows does not fill a 1 KiB DMA
            // block: such 2:4 tiles (BM <= 32) take the register pipeline
            // (the LDS allocated for PF holds its two stages)
            gemm_tile<BM, BN, WM, WN, FA, FB, SP, KFAST, 2, SWAP>(p, tm, tn, split, smem);
        } else {
            gemm_tile_dma<BM, BN, WM, WN, FA, FB, SP, PF - 4, PF, SWAP>(p, tm, tn, split, smem);
        }
        return;
    }
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    using S = TileSmem<BM, BN, SP, PF>;
    constexpr int A_CH = SP ? BM * 4 : BM * 8;     // 16-byte chunks per stage
    constexpr int M_CH = SP ? BM : 0;
    // a compressed j operand (SPB) loads 16-byte chunks of kept codes (32
    // dense positions each) plus their 4 metadata bytes and is expanded to
    // dense rows on its way into LDS
    constexpr int B_CH = SPB ? BN * 4 : BN * 8;
    constexpr int A_PER = (A_CH + NT - 1) / NT, B_PER = (B_CH + NT - 1) / NT;
    constexpr int M_PER = (M_CH + NT - 1) / NT;
    static_assert(PF >= 6 || ((A_CH % NT == 0 || A_CH < NT) && (B_CH % NT == 0 || B_CH < NT)),
                  "tile/thread mismatch");
    static_assert(TM >= 1 && TN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "wave tile");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lg = lane >> 4;
    const int m0 = tm * BM, n0 = tn * BN;
    const int kbeg = split * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);
    const int nk = (kend - kbeg + kBK - 1) / kBK;
    const int Kv = p.K / 2, Km = p.K / 8;   // compressed row lengths

    uint4 ra[PF][A_PER], rb[PF][B_PER], rm[PF][M_PER > 0 ? M_PER : 1];
    uint32_t rmb[PF][SPB ? B_PER : 1];

    // Chunks past the end of K are zeroed (metadata: given a valid filler)
    // when the registers are written to LDS, after the MFMAs of the step, so
    // the loads stay in flight across them.  Only a K that is not a multiple
    // of 16 (128 for compressed rows) takes the exact byte path instead.
    constexpr bool kfast = KFAST;
    // Fast path: buffer loads against per-tile resources whose range ends at
    // the last valid row, so rows past M or N read as zero and no access
    // leaves the operand; each thread needs one 32-bit offset per operand
    // and every further chunk is a uniform (scalar) offset from it.
    const int rows_a = min(BM, p.M - m0), rows_b = min(BN, p.N - n0);
    const __amdgpu_buffer_rsrc_t rs_a = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(p.a + (int64_t)m0 * p.lda), (short)0, rows_a * (int)p.lda, kBufferFlags);
    const __amdgpu_buffer_rsrc_t rs_b = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(p.b + (int64_t)n0 * p.ldb), (short)0, rows_b * (int)p.ldb, kBufferFlags);
    const __amdgpu_buffer_rsrc_t rs_m = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(SP ? p.meta + (int64_t)m0 * p.ldm : p.a), (short)0, SP ? rows_a * (int)p.ldm : 0, kBufferFlags);
    const int voff_a = SP ? (tid >> 2) * (int)p.lda + (tid & 3) * 16 : (tid >> 3) * (int)p.lda + (tid & 7) * 16;
    const int voff_b = SPB ? (tid >> 2) * (int)p.ldb + (tid & 3) * 16 : (tid >> 3) * (int)p.ldb + (tid & 7) * 16;
    const __amdgpu_buffer_rsrc_t rs_mb = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(SPB ? p.meta_b + (int64_t)n0 * p.ldmb : p.b), (short)0, SPB ? rows_b * (int)p.ldmb : 0,
        kBufferFlags);
    const int voff_mb = SPB ? (tid >> 2) * (int)p.ldmb + (tid & 3) * 4 : 0;
    const int voff_m = tid * (int)p.ldm;
    auto bload = [](const __amdgpu_buffer_rsrc_t &r, int voff, int soff) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        return make_uint4(v[0], v[1], v[2], v[3]);
    };
    auto gload = [&](int kt, uint4 *ra, uint4 *rb, uint4 *rm, uint32_t *rmb) {
        const int k0 = kbeg + kt * kBK;
        if constexpr (kfast) {
#pragma unroll
            for (int u = 0; u < A_PER; ++u) {
                if (A_CH < NT && tid + u * NT >= A_CH) break;
                ra[u] = SP ? bload(rs_a, voff_a, u * (NT / 4) * (int)p.lda + k0 / 2)
                           : bload(rs_a, voff_a, u * (NT / 8) * (int)p.lda + k0);
            }
            if constexpr (SP) {
#pragma unroll
                for (int u = 0; u < M_PER; ++u)
                    if (tid + u * NT < M_CH) rm[u] = bload(rs_m, voff_m, u * NT * (int)p.ldm + k0 / 8);
            }
#pragma unroll
            for (int u = 0; u < B_PER; ++u) {
                if (B_CH < NT && tid + u * NT >= B_CH) break;
                if constexpr (SPB) {
                    rb[u] = bload(rs_b, voff_b, u * (NT / 4) * (int)p.ldb + k0 / 2);
                    rmb[u] = __builtin_amdgcn_raw_buffer_load_b32(rs_mb, voff_mb, u * (NT / 4) * (int)p.ldmb + k0 / 8,
                                                                  0);
                } else {
                    rb[u] = bload(rs_b, voff_b, u * (NT / 8) * (int)p.ldb + k0);
                }
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_CH < NT && idx >= A_CH) break;
            if constexpr (SP) {
                const int r = idx >> 2, c = idx & 3;
                const int row = m0 + r;
                const int vk = k0 / 2 + c * 16;
                const uint8_t *src = p.a + (int64_t)(row < p.M ? row : 0) * p.lda;
                ra[u] = load16_partial(src + vk, row < p.M ? min(16, max(0, Kv - vk)) : 0, 0u);
            } else {
                const int r = idx >> 3, c = idx & 7;
                const int row = m0 + r;
                const int kk = k0 + c * 16;
                const uint8_t *src = p.a + (int64_t)(row < p.M ? row : 0) * p.lda;
                ra[u] = load16_partial(src + kk, row < p.M ? min(16, max(0, kend - kk)) : 0, 0u);
            }
        }
        if constexpr (SP) {
#pragma unroll
            for (int u = 0; u < M_PER; ++u) {
                const int r = tid + u * NT;
                if (r < M_CH) {
                    const int row = m0 + r;
                    const int mk = k0 / 8;
                    const uint8_t *src = p.meta + (int64_t)(row < p.M ? row : 0) * p.ldm;
                    rm[u] = load16_partial(src + mk, row < p.M ? min(16, max(0, Km - mk)) : 0, 0x44444444u);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_CH < NT && idx >= B_CH) break;
            if constexpr (SPB) {
                const int r = idx >> 2, c = idx & 3;
                const int row = n0 + r;
                const int vk = k0 / 2 + c * 16, mk = k0 / 8 + c * 4;
                const int64_t off = (int64_t)(row < p.N ? row : 0);
                rb[u] = load16_partial(p.b + off * p.ldb + vk, row < p.N ? min(16, max(0, Kv - vk)) : 0, 0u);
                uint32_t m = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (row < p.N && mk + t < Km) m |= (uint32_t)p.meta_b[off * p.ldmb + mk + t] << (8 * t);
                rmb[u] = m;
            } else {
                const int r = idx >> 3, c = idx & 7;
                const int row = n0 + r;
                const int kk = k0 + c * 16;
                const uint8_t *src = p.b + (int64_t)(row < p.N ? row : 0) * p.ldb;
                rb[u] = load16_partial(src + kk, row < p.N ? min(16, max(0, kend - kk)) : 0, 0u);
            }
        }
    };

    auto sel = [](const uint4 &v, bool ok, uint32_t fill) {
        return ok ? v : make_uint4(fill, fill, fill, fill);
    };

    auto sstore = [&](int buf, const uint4 *ra, const uint4 *rb, const uint4 *rm, const uint32_t *rmb, int kt) {
        const int k0 = kbeg + kt * kBK;
        uint8_t *base = smem + buf * S::STAGE;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_CH < NT && idx >= A_CH) break;
            if constexpr (SP) {
                const int r = idx >> 2, c = idx & 3;
                *reinterpret_cast<uint4 *>(base + swz_sp(r, c)) = kfast ? sel(ra[u], k0 / 2 + c * 16 < Kv, 0u) : ra[u];
            } else {
                const int r = idx >> 3, c = idx & 7;
                *reinterpret_cast<uint4 *>(base + swz(r, c)) = kfast ? sel(ra[u], k0 + c * 16 < kend, 0u) : ra[u];
            }
        }
        if constexpr (SP) {
#pragma unroll
            for (int u = 0; u < M_PER; ++u) {
                const int r = tid + u * NT;
                if (r < M_CH)
                    *reinterpret_cast<uint4 *>(base + S::A_BYTES + r * 16) =
                        kfast ? sel(rm[u], k0 / 8 < Km, 0x44444444u) : rm[u];
            }
        }
        uint8_t *bb = base + S::A_BYTES + S::M_BYTES;
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_CH < NT && idx >= B_CH) break;
            if constexpr (SPB) {
                // kept codes past the end of K (zeros) expand to zeros
                const int r = idx >> 2, c = idx & 3;
                uint4 d0, d1;
                expand24(kfast ? sel(rb[u], k0 / 2 + c * 16 < Kv, 0u) : rb[u], rmb[u], d0, d1);
                *reinterpret_cast<uint4 *>(bb + swz_b<SP>(r, 2 * c)) = d0;
                *reinterpret_cast<uint4 *>(bb + swz_b<SP>(r, 2 * c + 1)) = d1;
            } else {
                const int r = idx >> 3, c = idx & 7;
                *reinterpret_cast<uint4 *>(bb + swz_b<SP>(r, c)) = kfast ? sel(rb[u], k0 + c * 16 < kend, 0u) : rb[u];
            }
        }
    };

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    // One K step of MFMAs on LDS buffer `buf`.
    auto compute = [&](int buf) {
        const uint8_t *base = smem + buf * S::STAGE;
        const uint8_t *bb = base + S::A_BYTES + S::M_BYTES;
        // B fragment chunks: the dense instruction pairs lane group g of A and
        // B on codes 32g .. 32g+31; the sparse one expects B lane group g to
        // hold codes 16g .. 16g+15 and 64+16g .. 64+16g+15 of the step.
        const int bc0 = SP ? lg : 2 * lg, bc1 = SP ? lg + 4 : 2 * lg + 1;
        v8i bf[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int r = wn * WTN + j * 16 + lr;
            uint4 lo = *reinterpret_cast<const uint4 *>(bb + swz_b<SP>(r, bc0));
            uint4 hi = *reinterpret_cast<const uint4 *>(bb + swz_b<SP>(r, bc1));
            bf[j] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int r = wm * WTM + i * 16 + lr;
            if constexpr (SP) {
                uint4 v = *reinterpret_cast<const uint4 *>(base + swz_sp(r, lg));
                const int idx = *reinterpret_cast<const int *>(base + S::A_BYTES + r * 16 + lg * 4);
                v4i af = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma_sparse<FA, FB>(af, bf[j], acc[i][j], idx);
            } else {
                uint4 lo = *reinterpret_cast<const uint4 *>(base + swz(r, 2 * lg));
                uint4 hi = *reinterpret_cast<const uint4 *>(base + swz(r, 2 * lg + 1));
                v8i af = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                if constexpr (SWAP) {
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] = mfma_dense<FB, FA>(bf[j], af, acc[i][j]);
                } else {
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] = mfma_dense<FA, FB>(af, bf[j], acc[i][j]);
                }
            }
        }
    };

    if constexpr (PF == 3) {
        // Three LDS stages.  The B fragments and the first A fragment of step
        // k+1 are read from LDS into a second register set while the MFMAs
        // of step k run, so after each barrier a wave starts its MFMAs at
        // once; the other A fragments of a step are read from its own stage
        // while the previous row of MFMAs runs.  Step k: global loads of step
        // k+2 -> registers; MFMAs of step k; fragments of step k+1 <- stage
        // (k+1) % 3; registers -> stage (k+2) % 3 (last read during step
        // k-1, before the barrier that ended it); barrier.
        auto read_b = [&](int buf, v8i *gb) {
            const uint8_t *bb = smem + buf * S::STAGE + S::A_BYTES + S::M_BYTES;
            const int bc0 = SP ? lg : 2 * lg, bc1 = SP ? lg + 4 : 2 * lg + 1;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int r = wn * WTN + j * 16 + lr;
                uint4 lo = *reinterpret_cast<const uint4 *>(bb + swz_b<SP>(r, bc0));
                uint4 hi = *reinterpret_cast<const uint4 *>(bb + swz_b<SP>(r, bc1));
                gb[j] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
        };
        struct AFrag {
            v8i d;
            v4i s;
            int idx;
        };
        auto read_a = [&](int buf, int i) {
            const uint8_t *base = smem + buf * S::STAGE;
            const int r = wm * WTM + i * 16 + lr;
            AFrag f;
            if constexpr (SP) {
                uint4 v = *reinterpret_cast<const uint4 *>(base + swz_sp(r, lg));
                f.idx = *reinterpret_cast<const int *>(base + S::A_BYTES + r * 16 + lg * 4);
                f.s = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
            } else {
                uint4 lo = *reinterpret_cast<const uint4 *>(base + swz(r, 2 * lg));
                uint4 hi = *reinterpret_cast<const uint4 *>(base + swz(r, 2 * lg + 1));
                f.d = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
            }
            return f;
        };
        auto row_mma = [&](int i, const AFrag &f, const v8i *gb) {
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if constexpr (SP) acc[i][j] = mfma_sparse<FA, FB>(f.s, gb[j], acc[i][j], f.idx);
                else if constexpr (SWAP) acc[i][j] = mfma_dense<FB, FA>(gb[j], f.d, acc[i][j]);
                else acc[i][j] = mfma_dense<FA, FB>(f.d, gb[j], acc[i][j]);
            }
        };
        // MFMAs of the step held in stage `cur` (fragments gb, f0 already in
        // registers), then the next step's fragments from stage `nxt`.
        auto step = [&](int cur, const v8i *gb, const AFrag &f0, int nxt, v8i *nb, AFrag &n0) {
            row_mma(0, f0, gb);
#pragma unroll
            for (int i = 1; i < TM; ++i) row_mma(i, read_a(cur, i), gb);
            read_b(nxt, nb);
            n0 = read_a(nxt, 0);
        };
        v8i gb0[TN], gb1[TN];
        AFrag a0, a1;
        int s0 = 0, s1 = 1, s2 = 2;   // stages of steps k, k+1, k+2
        if (nk > 0) {
            gload(0, ra[0], rb[0], rm[0], rmb[0]);
            sstore(0, ra[0], rb[0], rm[0], rmb[0], 0);
            gload(1, ra[0], rb[0], rm[0], rmb[0]);
            sstore(1, ra[0], rb[0], rm[0], rmb[0], 1);
            __syncthreads();
            read_b(0, gb0);
            a0 = read_a(0, 0);
        }
        auto rot = [&]() {
            const int t = s0;
            s0 = s1;
            s1 = s2;
            s2 = t;
        };
        for (int kt = 0; kt < nk; kt += 2) {
            gload(kt + 2, ra[0], rb[0], rm[0], rmb[0]);
            step(s0, gb0, a0, s1, gb1, a1);
            sstore(s2, ra[0], rb[0], rm[0], rmb[0], kt + 2);
            __syncthreads();
            rot();
            if (kt + 1 >= nk) break;
            gload(kt + 3, ra[0], rb[0], rm[0], rmb[0]);
            step(s0, gb1, a1, s1, gb0, a0);
            sstore(s2, ra[0], rb[0], rm[0], rmb[0], kt + 3);
            __syncthreads();
            rot();
        }
    } else if constexpr (PF == 1) {
        // Loads of step k+1 go to the single register set during step k.
        if (nk > 0) {
            gload(0, ra[0], rb[0], rm[0], rmb[0]);
            sstore(0, ra[0], rb[0], rm[0], rmb[0], 0);
            __syncthreads();
        }
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) gload(kt + 1, ra[0], rb[0], rm[0], rmb[0]);
            compute(kt & 1);
            if (kt + 1 < nk) sstore((kt + 1) & 1, ra[0], rb[0], rm[0], rmb[0], kt + 1);
            __syncthreads();
        }
    } else {
        // Step k uses LDS buffer k % 2 and register set k % 2; the loop body
        // is written out for an even and an odd step so every register set
        // is named statically.  Loads and LDS stores are unconditional (past
        // the last step they read clamped, valid addresses and fill a buffer
        // nobody reads), which keeps the wait counts exact: the stores of a
        // step wait only for the loads issued a step earlier.
        if (nk > 0) {
            gload(0, ra[0], rb[0], rm[0], rmb[0]);
            gload(1, ra[PF - 1], rb[PF - 1], rm[PF - 1], rmb[PF - 1]);
            sstore(0, ra[0], rb[0], rm[0], rmb[0], 0);
            __syncthreads();
        }
        for (int kt = 0; kt < nk; kt += 2) {
            gload(kt + 2, ra[0], rb[0], rm[0], rmb[0]);
            compute(0);
            sstore(1, ra[PF - 1], rb[PF - 1], rm[PF - 1], rmb[PF - 1], kt + 1);
            __syncthreads();
            if (kt + 1 >= nk) break;
            gload(kt + 3, ra[PF - 1], rb[PF - 1], rm[PF - 1], rmb[PF - 1]);
            compute(1);
            sstore(0, ra[0], rb[0], rm[0], rmb[0], kt + 2);
            __syncthreads();
        }
    }

    // Epilogue.  With SWAP a lane holds four consecutive j of one i and a
    // row-major output takes them in one vector store; otherwise it holds four
    // consecutive i of one j, consecutive in memory when the output is stored
    // transposed (compressed weight, or a dense weight-major problem).
    static_assert(!(SP && SWAP), "the compressed operand must stay in the MFMA A slot");
    write_tile<BM, BN, WM, WN, SWAP, S::TOTAL>(p, acc, m0, n0, wave, lane, split, smem);
}

}  // namespace fp8k
