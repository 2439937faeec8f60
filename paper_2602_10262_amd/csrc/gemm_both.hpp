// GEMM with both operands 2:4-compressed along K (the both-side sparsity
// pattern of Sec. 7.1).  No gfx950 instruction takes two compressed operands:
// the i operand's kept codes feed the SMFMAC's compressed slot exactly as in
// the one-sided 2:4 GEMM, and the j operand's compressed rows (values and
// index nibbles) are expanded to dense rows in registers on their way into
// LDS, so the j operand crosses HBM at 0.625 bytes per element instead of 1.
// The exact-sum tiles expand both operands and sum on the BF16 MFMA.  Only the
// register-staged pipelines can expand (the DMA pipeline writes LDS without
// passing through registers), so the tiles below are a subset of the table.
#pragma once
#include "gemm_launch.hpp"

namespace fp8k {

// Tiles with a both-sides kernel (indices into the tile table).
#define FP8_BOTH_TILES(X) X(0) X(3) X(11) X(12) X(25) X(26) X(27)

template <int BM, int BN, int WM, int WN, int OCC, int PF, int FA, int FB, bool KFAST>
__global__ void __launch_bounds__(WM *WN * 64, OCC) gemm_both_kernel(GemmParams p)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileSmem<BM, BN, true, PF>::TOTAL];
    int tm, tn;
    tile_coords<BM, BN>(p.M, p.N, tm, tn);
    gemm_tile<BM, BN, WM, WN, FA, FB, true, KFAST, PF, false, true>(p, tm, tn, blockIdx.z, smem);
}

template <int BM, int BN, int WM, int WN, int OCC, int PF, bool KFAST>
hipError_t launch_both_one(int fa, int fb, const GemmParams &p, hipStream_t st)
{
    static_assert(PF <= 3 || PF == kExactPF, "register-staged pipelines only");
    static_assert(tile_sparse_ok(BM) || PF == kExactPF, "2:4 tile");
    const int nb = ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN);
    dim3 grid((unsigned)nb, 1, (unsigned)p.splits), block(WM * WN * 64);
#define FP8_GO(FA, FB) gemm_both_kernel<BM, BN, WM, WN, OCC, PF, FA, FB, KFAST><<<grid, block, 0, st>>>(p)
    switch (fa * 2 + fb) {
    case 0: FP8_GO(0, 0); break;
    case 1: FP8_GO(0, 1); break;
    case 2: FP8_GO(1, 0); break;
    default: FP8_GO(1, 1); break;
    }
#undef FP8_GO
    return hipGetLastError();
}

template <int T>
hipError_t launch_both_tile(int fa, int fb, const GemmParams &p, hipStream_t st)
{
    using C = TileCfg<T>;
    if constexpr (C::PF == kExactPF) {
        if (!k_is_fast(true, p.K)) return launch_both_one<C::BM, C::BN, C::WM, C::WN, C::OCC, C::PF, false>(fa, fb, p, st);
    }
    return launch_both_one<C::BM, C::BN, C::WM, C::WN, C::OCC, C::PF, true>(fa, fb, p, st);
}
#define FP8_BOTH_EXTERN(i) extern template hipError_t launch_both_tile<i>(int, int, const GemmParams &, hipStream_t);
FP8_BOTH_TILES(FP8_BOTH_EXTERN)
#undef FP8_BOTH_EXTERN
#define FP8_BOTH_INSTANTIATE(i) template hipError_t launch_both_tile<i>(int, int, const GemmParams &, hipStream_t);

}  // namespace fp8k
