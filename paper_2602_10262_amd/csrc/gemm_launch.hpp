// The plain/split-K GEMM kernel and its per-tile launcher, shared by the
// translation units that instantiate the tile table (split over several
// files so that they compile in parallel).
//
// Workgroup -> tile mapping: the hardware hands workgroups to the 8 XCDs
// round robin, so workgroup b is first renumbered so that each XCD receives a
// contiguous run of tile numbers; the runs are then laid out in groups of
// kGroupM tile rows (column-major inside a group) so that the workgroups an
// XCD runs together share A rows and B columns in its L2.
#pragma once
#include "gemm_tile.hpp"

namespace fp8k {

constexpr int kGroupM = 8;
constexpr int kXcds = 8;

template <int BM, int BN>
__device__ __forceinline__ void tile_coords(int M, int N, int &tm, int &tn)
{
    const int nbm = (M + BM - 1) / BM, nbn = (N + BN - 1) / BN;
    const int nb = nbm * nbn;
    int bid = blockIdx.x;
    if (nb % kXcds == 0) bid = (bid % kXcds) * (nb / kXcds) + bid / kXcds;
    const int per_group = kGroupM * nbn;
    const int g = bid / per_group;
    const int first = g * kGroupM;
    const int rows_in_group = min(nbm - first, kGroupM);
    const int in = bid % per_group;
    tm = first + in % rows_in_group;
    tn = in / rows_in_group;
}

template <int BM, int BN, int WM, int WN, int OCC, int PF, int FA, int FB, bool SP, bool KFAST>
__global__ void __launch_bounds__(WM *WN * 64, OCC) gemm_kernel(GemmParams p)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileSmem<BM, BN, SP, PF>::TOTAL];
    int tm, tn;
    tile_coords<BM, BN>(p.M, p.N, tm, tn);
    gemm_tile<BM, BN, WM, WN, FA, FB, SP, KFAST, PF>(p, tm, tn, blockIdx.z, smem);
}

template <int BM, int BN, int WM, int WN, int OCC, int PF, bool KFAST = true>
hipError_t launch_one(int fa, int fb, bool sp, const GemmParams &p, hipStream_t st)
{
    const int nb = ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN);
    dim3 grid((unsigned)nb, 1, (unsigned)p.splits), block(WM * WN * 64);
#define FP8_GO(FA, FB, SP) gemm_kernel<BM, BN, WM, WN, OCC, PF, FA, FB, SP, KFAST><<<grid, block, 0, st>>>(p)
    constexpr bool DENSE = tile_dense_fits(BM, BN, PF);
    constexpr bool SPARSE = (tile_sparse_ok(BM) || PF == kExactPF) && !pf_mfma32(PF);
    // (plan resolution rejects a dense or 2:4 request for a tile without that kernel)
    if (sp) {
        if constexpr (SPARSE) {
            switch (fa * 2 + fb) {
            case 0: FP8_GO(0, 0, true); break;
            case 1: FP8_GO(0, 1, true); break;
            case 2: FP8_GO(1, 0, true); break;
            default: FP8_GO(1, 1, true); break;
            }
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        if constexpr (DENSE) {
            switch (fa * 2 + fb) {
            case 0: FP8_GO(0, 0, false); break;
            case 1: FP8_GO(0, 1, false); break;
            case 2: FP8_GO(1, 0, false); break;
            default: FP8_GO(1, 1, false); break;
            }
        } else {
            return hipErrorInvalidValue;
        }
    }
#undef FP8_GO
    return hipGetLastError();
}


// Parameters of tile T of the table.
template <int T>
struct TileCfg;
#define FP8_CFG(i, bm, bn, wm, wn, occ, pf)                                                  \
    template <>                                                                           \
    struct TileCfg<i> {                                                                   \
        static constexpr int BM = bm, BN = bn, WM = wm, WN = wn, OCC = occ, PF = pf;      \
    };
FP8_TILE_LIST(FP8_CFG)
#undef FP8_CFG

// Launches tile T.  Each T is instantiated in exactly one gemm_tiles_*.hip
// file (declared extern here so that no other file compiles it again).
template <int T>
hipError_t launch_tile(int fa, int fb, bool sp, const GemmParams &p, hipStream_t st)
{
    using C = TileCfg<T>;
    // an exact-sum tile loads byte-exact itself when K leaves partial chunks;
    // the exact-sum DMA tiles hand such a K to the tile that does
    if constexpr (C::PF == kExactPF) {
        if (!k_is_fast(sp, p.K)) return launch_one<C::BM, C::BN, C::WM, C::WN, C::OCC, C::PF, false>(fa, fb, sp, p, st);
    } else if constexpr (pf_exact_dma(C::PF)) {
        if (!k_is_fast(sp, p.K)) return launch_tile<kExactAnyKTile>(fa, fb, sp, p, st);
    }
    return launch_one<C::BM, C::BN, C::WM, C::WN, C::OCC, C::PF>(fa, fb, sp, p, st);
}
#define FP8_EXTERN(i, bm, bn, wm, wn, occ, pf) \
    extern template hipError_t launch_tile<i>(int, int, bool, const GemmParams &, hipStream_t);
FP8_TILE_LIST(FP8_EXTERN)
#undef FP8_EXTERN
#define FP8_INSTANTIATE(i) template hipError_t launch_tile<i>(int, int, bool, const GemmParams &, hipStream_t);

}  // namespace fp8k
