// Plain and split-K FP8 GEMM launches on gfx950 (dense and 2:4), plus the
// fixed-order split-K reduction.
//
// Workgroup -> tile mapping: the hardware hands workgroups to the 8 XCDs
// round robin, so workgroup b is first renumbered so that each XCD receives a
// contiguous run of tile numbers; the runs are then laid out in groups of
// kGroupM tile rows (column-major inside a group) so that the workgroups an
// XCD runs together share A rows and B columns in its L2.
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

#define FP8_DESC(i, bm, bn, wm, wn, occ, pf) {bm, bn, wm * wn, 1},
static const TileDesc kTiles[] = {FP8_TILE_LIST(FP8_DESC)};
#undef FP8_DESC

int num_tiles() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileDesc &tile_desc(int t) { return kTiles[t]; }

template <int BM, int BN, int WM, int WN, int OCC, int PF, bool KFAST = true>
static hipError_t launch_one(int fa, int fb, bool sp, const GemmParams &p, hipStream_t st)
{
    const int nb = ((p.M + BM - 1) / BM) * ((p.N + BN - 1) / BN);
    dim3 grid((unsigned)nb, 1, (unsigned)p.splits), block(WM * WN * 64);
#define FP8_GO(FA, FB, SP) gemm_kernel<BM, BN, WM, WN, OCC, PF, FA, FB, SP, KFAST><<<grid, block, 0, st>>>(p)
    const int key = fa * 4 + fb * 2 + (sp ? 1 : 0);
    switch (key) {
    case 0: FP8_GO(0, 0, false); break;
    case 1: FP8_GO(0, 0, true); break;
    case 2: FP8_GO(0, 1, false); break;
    case 3: FP8_GO(0, 1, true); break;
    case 4: FP8_GO(1, 0, false); break;
    case 5: FP8_GO(1, 0, true); break;
    case 6: FP8_GO(1, 1, false); break;
    default: FP8_GO(1, 1, true); break;
    }
#undef FP8_GO
    return hipGetLastError();
}

bool k_is_fast(bool sparse, int K) { return sparse ? (K % 128) == 0 : (K % 16) == 0; }

hipError_t launch_gemm(int tile, int fa, int fb, bool sparse, const GemmParams &p, hipStream_t st)
{
    // A K that leaves partial 16-byte chunks runs on the byte-exact loader,
    // compiled for the 128 x 128 tile only.
    if (!k_is_fast(sparse, p.K)) return launch_one<128, 128, 2, 2, 1, 1, false>(fa, fb, sparse, p, st);
    switch (tile) {
#define FP8_CASE(i, bm, bn, wm, wn, occ, pf) \
    case i: return launch_one<bm, bn, wm, wn, occ, pf>(fa, fb, sparse, p, st);
        FP8_TILE_LIST(FP8_CASE)
#undef FP8_CASE
    default: return hipErrorInvalidValue;
    }
}

// C = ((sum over splits in order) * descale...) from the [splits][M][N] workspace.
__global__ void __launch_bounds__(256) splitk_reduce(GemmParams p)
{
    const int64_t total = (int64_t)p.M * p.N;
    const int64_t plane = total;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        float acc = 0.0f;
        for (int s = 0; s < p.splits; ++s) acc += p.ws[s * plane + t];
        store_out(p, (int)(t / p.N), (int)(t % p.N), acc);
    }
}

hipError_t launch_splitk_reduce(const GemmParams &p, hipStream_t st)
{
    const int64_t total = (int64_t)p.M * p.N;
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    splitk_reduce<<<(unsigned)(g < 1 ? 1 : g), 256, 0, st>>>(p);
    return hipGetLastError();
}

}  // namespace fp8k
