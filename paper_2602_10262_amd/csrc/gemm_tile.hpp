// The FP8 GEMM macro-tile shared by the plain, split-K and grouped kernels.
//
// One workgroup computes a BM x BN block of C over a K range, in steps of 128
// codes of K:
//   - stage loads: 128-bit global loads of the next step's A and B tiles are
//     issued into registers before the current step's MFMAs and written to
//     the other half of a double-buffered LDS area after them, so one
//     barrier per step suffices;
//   - LDS layout: dense operands keep one 128-byte row per tile row, the
//     sixteen-byte chunks of row r permuted by XOR with (r >> 1) & 7 so that
//     the sixteen rows a fragment read touches spread over all banks;
//     compressed operands keep 64 value bytes and 16 metadata bytes per row;
//   - each wave owns a (BM / WM) x (BN / WN) sub-block made of 16 x 16
//     accumulators; per step it reads its A and B fragments from LDS and
//     issues v_mfma_f32_16x16x128_f8f6f4 (dense: lane l supplies row l % 16,
//     codes 32 (l / 16) .. 32 (l / 16) + 31 of the step, for both operands)
//     or v_smfmac_f32_16x16x128_* (2:4: lane l supplies the 16 survivors of
//     those 32 positions and their eight index nibbles as one 32-bit word,
//     while its B lane holds codes 16 (l / 16) + 0..15 and 64 + 16 (l / 16)
//     + 0..15, the layout the sparse instruction pairs with);
//   - epilogue: descales applied in FP32, C stored as FP32 or BF16 (RNE), or
//     raw FP32 partial sums to the split-K workspace.
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace fp8k {

constexpr int kBK = 128;

template <int BM, int BN, bool SP>
struct TileSmem {
    static constexpr int A_BYTES = SP ? BM * 64 : BM * 128;
    static constexpr int M_BYTES = SP ? BM * 16 : 0;
    static constexpr int B_BYTES = BN * 128;
    static constexpr int STAGE = A_BYTES + M_BYTES + B_BYTES;
    static constexpr int TOTAL = 2 * STAGE;
};

__device__ __forceinline__ int swz(int r, int c) { return (r * 128) + ((c ^ ((r >> 1) & 7)) << 4); }

// 16 bytes from global memory; `valid` (0..16) leading bytes are real, the
// rest take `fill`.
__device__ __attribute__((noinline)) uint4 load16_partial(const uint8_t *p, int valid, uint32_t fill)
{
    uint32_t w[4] = {fill, fill, fill, fill};
    for (int b = 0; b < valid && b < 16; ++b) {
        w[b / 4] &= ~(0xFFu << (8 * (b % 4)));
        w[b / 4] |= (uint32_t)p[b] << (8 * (b % 4));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint4 load16(const uint8_t *p, int valid, uint32_t fill)
{
    if (valid >= 16) return *reinterpret_cast<const uint4 *>(p);
    return load16_partial(p, valid, fill);
}

// The same for a source whose rows need not be 16-byte aligned (compressed
// rows of K/2 and K/8 bytes when K is not a multiple of 128).
__device__ __forceinline__ uint4 load16_any(const uint8_t *p, int valid, uint32_t fill)
{
    if (valid >= 16 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) return *reinterpret_cast<const uint4 *>(p);
    return load16_partial(p, valid, fill);
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
    else reinterpret_cast<float *>(p.c)[off] = v;
}

// Computes tile (tm, tn) of split `split`.  smem: TileSmem<BM,BN,SP>::TOTAL bytes.
template <int BM, int BN, int WM, int WN, int FA, int FB, bool SP>
__device__ __forceinline__ void gemm_tile(const GemmParams &p, int tm, int tn, int split, uint8_t *smem)
{
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    using S = TileSmem<BM, BN, SP>;
    constexpr int A_CH = SP ? BM * 4 : BM * 8;     // 16-byte chunks per stage
    constexpr int M_CH = SP ? BM : 0;
    constexpr int B_CH = BN * 8;
    constexpr int A_PER = (A_CH + NT - 1) / NT, B_PER = (B_CH + NT - 1) / NT;
    constexpr int M_PER = (M_CH + NT - 1) / NT;
    static_assert((A_CH % NT == 0 || A_CH < NT) && (B_CH % NT == 0 || B_CH < NT), "tile/thread mismatch");
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

    uint4 ra[A_PER], rb[B_PER], rm[M_PER > 0 ? M_PER : 1];

    auto gload = [&](int kt) {
        const int k0 = kbeg + kt * kBK;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_CH < NT && idx >= A_CH) break;
            if constexpr (SP) {
                const int r = idx >> 2, c = idx & 3;
                const int row = m0 + r;
                const int vk = k0 / 2 + c * 16;
                const int valid = row < p.M ? min(16, max(0, Kv - vk)) : 0;
                ra[u] = load16_any(p.a + (int64_t)(row < p.M ? row : 0) * p.lda + (valid > 0 ? vk : 0), valid, 0u);
            } else {
                const int r = idx >> 3, c = idx & 7;
                const int row = m0 + r;
                const int kk = k0 + c * 16;
                const int valid = row < p.M ? min(16, max(0, kend - kk)) : 0;
                ra[u] = load16(p.a + (int64_t)(row < p.M ? row : 0) * p.lda + (valid > 0 ? kk : 0), valid, 0u);
            }
        }
        if constexpr (SP) {
#pragma unroll
            for (int u = 0; u < M_PER; ++u) {
                const int r = tid + u * NT;
                if (r < M_CH) {
                    const int row = m0 + r;
                    const int mk = k0 / 8;
                    const int valid = row < p.M ? min(16, max(0, Km - mk)) : 0;
                    rm[u] = load16_any(p.meta + (int64_t)(row < p.M ? row : 0) * p.ldm + (valid > 0 ? mk : 0), valid,
                                   0x44444444u);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_CH < NT && idx >= B_CH) break;
            const int r = idx >> 3, c = idx & 7;
            const int row = n0 + r;
            const int kk = k0 + c * 16;
            const int valid = row < p.N ? min(16, max(0, kend - kk)) : 0;
            rb[u] = load16(p.b + (int64_t)(row < p.N ? row : 0) * p.ldb + (valid > 0 ? kk : 0), valid, 0u);
        }
    };

    auto sstore = [&](int buf) {
        uint8_t *base = smem + buf * S::STAGE;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_CH < NT && idx >= A_CH) break;
            if constexpr (SP) {
                *reinterpret_cast<uint4 *>(base + idx * 16) = ra[u];
            } else {
                const int r = idx >> 3, c = idx & 7;
                *reinterpret_cast<uint4 *>(base + swz(r, c)) = ra[u];
            }
        }
        if constexpr (SP) {
#pragma unroll
            for (int u = 0; u < M_PER; ++u) {
                const int r = tid + u * NT;
                if (r < M_CH) *reinterpret_cast<uint4 *>(base + S::A_BYTES + r * 16) = rm[u];
            }
        }
        uint8_t *bb = base + S::A_BYTES + S::M_BYTES;
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_CH < NT && idx >= B_CH) break;
            const int r = idx >> 3, c = idx & 7;
            *reinterpret_cast<uint4 *>(bb + swz(r, c)) = rb[u];
        }
    };

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    if (nk > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
    }
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kt + 1);
        const uint8_t *base = smem + cur * S::STAGE;
        const uint8_t *bb = base + S::A_BYTES + S::M_BYTES;
        // B fragment chunks: the dense instruction pairs lane group g of A and
        // B on codes 32g .. 32g+31; the sparse one expects B lane group g to
        // hold codes 16g .. 16g+15 and 64+16g .. 64+16g+15 of the step.
        const int bc0 = SP ? lg : 2 * lg, bc1 = SP ? lg + 4 : 2 * lg + 1;
        v8i bf[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int r = wn * WTN + j * 16 + lr;
            uint4 lo = *reinterpret_cast<const uint4 *>(bb + swz(r, bc0));
            uint4 hi = *reinterpret_cast<const uint4 *>(bb + swz(r, bc1));
            bf[j] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int r = wm * WTM + i * 16 + lr;
            if constexpr (SP) {
                uint4 v = *reinterpret_cast<const uint4 *>(base + r * 64 + lg * 16);
                const int idx = *reinterpret_cast<const int *>(base + S::A_BYTES + r * 16 + lg * 4);
                v4i af = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma_sparse<FA, FB>(af, bf[j], acc[i][j], idx);
            } else {
                uint4 lo = *reinterpret_cast<const uint4 *>(base + swz(r, 2 * lg));
                uint4 hi = *reinterpret_cast<const uint4 *>(base + swz(r, 2 * lg + 1));
                v8i af = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = mfma_dense<FA, FB>(af, bf[j], acc[i][j]);
            }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    // epilogue: lane holds rows 4*lg .. 4*lg+3 of column lr of each 16 x 16 accumulator
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int col = n0 + wn * WTN + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * WTM + i * 16 + 4 * lg + r;
                if (row < p.M && col < p.N) {
                    if (p.splits > 1)
                        p.ws[((int64_t)split * p.M + row) * p.N + col] = acc[i][j][r];
                    else
                        store_out(p, row, col, acc[i][j][r]);
                }
            }
        }
}

}  // namespace fp8k
