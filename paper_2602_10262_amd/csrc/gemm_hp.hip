// FP32, FP16 and BF16 GEMMs: the higher-precision stages of the
// mixed-precision sequence (Sec. 8.3: FP32 and 16-bit matrix operations run
// beside the FP8 ones), on gfx950's matrix cores:
//   FP32: v_mfma_f32_16x16x4_f32 (products and sums in FP32),
//   FP16 / BF16: v_mfma_f32_16x16x32_f16 / _bf16 (exact products, FP32 sums).
// Same operand convention as the FP8 GEMM: A row-major M x K, B as N rows of
// K (column-major K x N), C = (acc * s_a[i]) * s_b[j] stored as FP32, BF16 or
// FP16 by the FP8 GEMM's epilogue.  Leading dimensions count elements.
//
// Pipelines: 256 x 256 with 8 waves on the FP8 tiles' two-stage LDS-DMA
// ring (128-byte rows: 32 FP32 or 64 16-bit elements of K per step) when K
// fills whole 16-byte chunks; otherwise two LDS stages with the loads of step
// k + 1 staged in registers during the MFMAs of step k: 256 x 256 with 8
// waves on 128-byte rows, 128 x 128 and 64 x 64 with 4 waves on 256-byte
// rows (64 or 128 elements).
// Lane l reads row l % 16 at chunk 4 s + l / 16 for sub-step s: 8 elements of
// K for the 16-bit instruction (its K = 32 per sub-step), 4 for FP32, where
// instruction t of the sub-step takes element t of every lane's chunk (any
// assignment of K to instructions works as long as A and B agree).
#include <cstring>
#include <string>

#include "api_util.hpp"
#include "gemm_launch.hpp"

namespace fp8k {

namespace {

// RB: bytes of K per LDS row and step (256: chunk x of row r at x ^ (r & 15);
// 128: the 2:4 kernels' B swizzle, conflict-free for chunk positions (g, g+4)).
template <int BM, int BN, int RB>
struct HpSmem {
    static constexpr int STAGE = (BM + BN) * RB;
    static constexpr int TOTAL = 2 * STAGE;
};

template <int RB>
__device__ __forceinline__ int hp_slot(int r, int x)
{
    if constexpr (RB == 256) return r * 256 + ((x ^ (r & 15)) << 4);
    else return swz_b2(r, x);
}

template <int BM, int BN, int WM, int WN, int T, int RB>
__device__ __forceinline__ void gemm_tile_hp(const GemmParams &p, int tm, int tn, uint8_t *smem)
{
    constexpr int ES = T == kHpF32 ? 4 : 2;
    constexpr int KS = RB / ES;
    constexpr int CH = RB / 16;            // 16-byte chunks per row and step
    constexpr int SUB = RB / 64;           // sub-steps (four chunk positions each)
    constexpr int NT = WM * WN * 64;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 16, TN = WTN / 16;
    constexpr int A_U = BM * CH, B_U = BN * CH;
    constexpr int A_PER = (A_U + NT - 1) / NT, B_PER = (B_U + NT - 1) / NT;
    using S = HpSmem<BM, BN, RB>;
    static_assert(TM >= 1 && TN >= 1, "wave tile");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int lr = lane & 15, lg = lane >> 4;
    const int m0 = tm * BM, n0 = tn * BN;
    const int nk = (p.K + KS - 1) / KS;
    const int rowbytes = p.K * ES;

    uint4 ra[A_PER], rb[B_PER];
    auto gload = [&](int kt) {
        const int kb = kt * KS * ES;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_U % NT != 0 && idx >= A_U) break;
            const int r = idx / CH, c = idx % CH, row = m0 + r;
            ra[u] = row < p.M ? load_codes16(p.a + (int64_t)row * p.lda * ES, kb + 16 * c, rowbytes)
                              : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_U % NT != 0 && idx >= B_U) break;
            const int r = idx / CH, c = idx % CH, row = n0 + r;
            rb[u] = row < p.N ? load_codes16(p.b + (int64_t)row * p.ldb * ES, kb + 16 * c, rowbytes)
                              : make_uint4(0, 0, 0, 0);
        }
    };
    auto put = [&](uint8_t *base, int r, int x, const uint4 &v) {
        *reinterpret_cast<uint4 *>(base + hp_slot<RB>(r, x)) = v;
    };
    auto sstore = [&](int buf) {
        uint8_t *base = smem + buf * S::STAGE;
#pragma unroll
        for (int u = 0; u < A_PER; ++u) {
            const int idx = tid + u * NT;
            if (A_U % NT != 0 && idx >= A_U) break;
            put(base, idx / CH, idx % CH, ra[u]);
        }
        uint8_t *bb = base + BM * RB;
#pragma unroll
        for (int u = 0; u < B_PER; ++u) {
            const int idx = tid + u * NT;
            if (B_U % NT != 0 && idx >= B_U) break;
            put(bb, idx / CH, idx % CH, rb[u]);
        }
    };

    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

    auto chunk = [&](const uint8_t *base, int r, int x) {
        return *reinterpret_cast<const uint4 *>(base + hp_slot<RB>(r, x));
    };
    auto compute = [&](int buf) {
        const uint8_t *base = smem + buf * S::STAGE;
        const uint8_t *bb = base + BM * RB;
#pragma unroll
        for (int s = 0; s < SUB; ++s) {
            uint4 bf[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = chunk(bb, wn * WTN + j * 16 + lr, 4 * s + lg);
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const uint4 af = chunk(base, wm * WTM + i * 16 + lr, 4 * s + lg);
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if constexpr (T == kHpF32) {
                        const uint32_t a4[4] = {af.x, af.y, af.z, af.w};
                        const uint32_t b4[4] = {bf[j].x, bf[j].y, bf[j].z, bf[j].w};
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a4[t]),
                                                                             __uint_as_float(b4[t]), acc[i][j], 0, 0,
                                                                             0);
                    } else if constexpr (T == kHpF16) {
                        typedef _Float16 v8h __attribute__((ext_vector_type(8)));
                        v8h a8, b8;
                        __builtin_memcpy(&a8, &af, 16);
                        __builtin_memcpy(&b8, &bf[j], 16);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a8, b8, acc[i][j], 0, 0, 0);
                    } else {
                        typedef __bf16 v8b __attribute__((ext_vector_type(8)));
                        v8b a8, b8;
                        __builtin_memcpy(&a8, &af, 16);
                        __builtin_memcpy(&b8, &bf[j], 16);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b8, acc[i][j], 0, 0, 0);
                    }
                }
            }
        }
    };

    if (nk > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) gload(kt + 1);
            compute(kt & 1);
            if (kt + 1 < nk) sstore((kt + 1) & 1);
            __syncthreads();
        }
    }
    write_tile<BM, BN, WM, WN, false, S::TOTAL>(p, acc, m0, n0, wave, lane, 0, smem);
}

template <int BM, int BN, int WM, int WN, int OCC, int T, int RB>
__global__ void __launch_bounds__(WM *WN * 64, OCC) gemm_hp_kernel(GemmParams p)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[HpSmem<BM, BN, RB>::TOTAL];
    int tm, tn;
    tile_coords<BM, BN>(p.M, p.N, tm, tn);
    gemm_tile_hp<BM, BN, WM, WN, T, RB>(p, tm, tn, smem);
}

// The 256 x 256 tile on the FP8 tiles' LDS-DMA ring (two stages of 128-byte
// rows, no staging registers); p counts K and the leading dimensions in bytes.
template <int T>
__global__ void __launch_bounds__(512, 1) gemm_hp_dma_kernel(GemmParams p)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileSmem<256, 256, false, 6>::TOTAL];
    int tm, tn;
    tile_coords<256, 256>(p.M, p.N, tm, tn);
    gemm_tile_dma<256, 256, 2, 4, 0, 0, false, 2, 6, true, T>(p, tm, tn, 0, smem);
}

hipError_t launch_hp_dma(int t, const GemmParams &p, int es, hipStream_t st)
{
    GemmParams q = p;
    q.K = p.K * es;
    q.lda = p.lda * es;
    q.ldb = p.ldb * es;
    q.kchunk = (q.K + kBK - 1) / kBK * kBK;
    const int nb = ((p.M + 255) / 256) * ((p.N + 255) / 256);
    const dim3 grid((unsigned)nb), block(512);
    if (t == kHpF32) gemm_hp_dma_kernel<kHpF32><<<grid, block, 0, st>>>(q);
    else if (t == kHpF16) gemm_hp_dma_kernel<kHpF16><<<grid, block, 0, st>>>(q);
    else gemm_hp_dma_kernel<kHpBF16><<<grid, block, 0, st>>>(q);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int OCC, int RB>
hipError_t launch_hp(int t, const GemmParams &p, hipStream_t st)
{
    const int nb = ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN);
    const dim3 grid((unsigned)nb), block(WM * WN * 64);
    if (t == kHpF32) gemm_hp_kernel<BM, BN, WM, WN, OCC, kHpF32, RB><<<grid, block, 0, st>>>(p);
    else if (t == kHpF16) gemm_hp_kernel<BM, BN, WM, WN, OCC, kHpF16, RB><<<grid, block, 0, st>>>(p);
    else gemm_hp_kernel<BM, BN, WM, WN, OCC, kHpBF16, RB><<<grid, block, 0, st>>>(p);
    return hipGetLastError();
}

bool aligned16(const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; }

}  // namespace

// Tile choice: 256 x 256 (8 waves, 128-byte rows) once there are enough
// such tiles for the chip, then 128 x 128 (4 waves), else 64 x 64.
int hp_tile_rows(int64_t M, int64_t N)
{
    if (((M + 255) / 256) * ((N + 255) / 256) >= 256) return 256;
    return ((M + 127) / 128) * ((N + 127) / 128) >= 256 ? 128 : 64;
}

}  // namespace fp8k

using namespace fp8k;

extern "C" {

fp8_status fp8_hp_gemm(const fp8_hp_gemm_args *a, void *stream)
{
    if (!a) return set_error(FP8_ERR_ARG, "null args");
    if (a->M < 1 || a->N < 1 || a->K < 1 || a->M > (1 << 30) || a->N > (1 << 30) || a->K > (1 << 20))
        return set_error(FP8_ERR_SHAPE, "M, N in [1, 2^30], K in [1, 2^20]");
    if (a->ab_type != FP8_HP_F32 && a->ab_type != FP8_HP_F16 && a->ab_type != FP8_HP_BF16)
        return set_error(FP8_ERR_ARG, "unknown operand type");
    if (a->c_type != FP8_OUT_F32 && a->c_type != FP8_OUT_BF16 && a->c_type != FP8_OUT_F16)
        return set_error(FP8_ERR_ARG, "unknown output type");
    if ((a->a_kind != FP8_SCALE_TENSOR && a->a_kind != FP8_SCALE_ROW) ||
        (a->b_kind != FP8_SCALE_TENSOR && a->b_kind != FP8_SCALE_ROW))
        return set_error(FP8_ERR_ARG, "unknown scale kind");
    if (!a->a || !a->b || !a->c || !a->a_scale || !a->b_scale) return set_error(FP8_ERR_ARG, "null pointer");
    if (a->tile_rows != 0 && a->tile_rows != 64 && a->tile_rows != 128 && a->tile_rows != 256)
        return set_error(FP8_ERR_ARG, "tile_rows must be 0, 64, 128 or 256");
    if (a->lda < a->K || a->ldb < a->K || a->ldc < a->N) return set_error(FP8_ERR_ARG, "leading dimension too small");
    const int es = a->ab_type == FP8_HP_F32 ? 4 : 2;
    if ((int64_t)256 * a->lda * es >= ((int64_t)1 << 31) || (int64_t)256 * a->ldb * es >= ((int64_t)1 << 31))
        return set_error(FP8_ERR_SHAPE, "leading dimensions too large");
    if (!aligned16(a->a) || !aligned16(a->b) || (a->lda * es) % 16 || (a->ldb * es) % 16)
        return set_error(FP8_ERR_ALIGN, "A and B must be 16-byte aligned with 16-byte row strides");
    GemmParams p;
    std::memset(&p, 0, sizeof(p));
    p.a = static_cast<const uint8_t *>(a->a); p.lda = a->lda;
    p.b = static_cast<const uint8_t *>(a->b); p.ldb = a->ldb;
    p.si = a->a_scale; p.si_per = a->a_kind == FP8_SCALE_ROW;
    p.sj = a->b_scale; p.sj_per = a->b_kind == FP8_SCALE_ROW;
    p.c = a->c; p.ldc = a->ldc;
    p.out_bf16 = a->c_type == FP8_OUT_BF16;
    p.out_f16 = a->c_type == FP8_OUT_F16;
    p.M = (int)a->M; p.N = (int)a->N; p.K = (int)a->K;
    p.splits = 1;
    p.kchunk = p.K;
    const int t = a->ab_type == FP8_HP_F32 ? 0 : (a->ab_type == FP8_HP_F16 ? 1 : 2);
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int rows = a->tile_rows > 0 ? a->tile_rows : hp_tile_rows(a->M, a->N);
    hipError_t e;
    // the DMA ring needs K in whole 16-byte chunks; other K take the
    // register-staged 256 x 256 tile
    if (rows == 256 && (p.K * es) % 16 == 0) e = launch_hp_dma(t, p, es, st);
    else if (rows == 256) e = launch_hp<256, 256, 2, 4, 1, 128>(t, p, st);
    else if (rows == 128) e = launch_hp<128, 128, 2, 2, 1, 256>(t, p, st);
    else e = launch_hp<64, 64, 2, 2, 2, 256>(t, p, st);
    if (e != hipSuccess) return hip_error(e, "higher-precision gemm launch");
    return FP8_OK;
}

}  // extern "C"
