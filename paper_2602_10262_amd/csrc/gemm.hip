// Plain and split-K FP8 GEMM launches on gfx950 (dense and 2:4): tile table,
// dispatch, the byte-exact kernel for K with partial 16-byte chunks, and the
// fixed-order split-K reduction.  The tile kernels themselves are
// instantiated in gemm_tiles_*.hip.
#include "gemm_launch.hpp"

namespace fp8k {

#define FP8_DESC(i, bm, bn, wm, wn, occ, pf)                                                     \
    {bm, bn, wm * wn, ((tile_sparse_ok(bm) || pf == kExactPF) && !pf_mfma32(pf)) ? 1 : 0, pf_exact(pf) ? 1 : 0, \
     tile_dense_fits(bm, bn, pf) ? 1 : 0},
static const TileDesc kTiles[] = {FP8_TILE_LIST(FP8_DESC)};
#undef FP8_DESC

int num_tiles() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileDesc &tile_desc(int t) { return kTiles[t]; }

bool k_is_fast(bool sparse, int K) { return sparse ? (K % 128) == 0 : (K % 16) == 0; }

hipError_t launch_gemm(int tile, int fa, int fb, bool sparse, const GemmParams &p, hipStream_t st)
{
    // A K that leaves partial 16-byte chunks runs on the byte-exact loader,
    // compiled for the 128 x 128 tile only.
    // (the exact-sum tiles load byte-exact themselves)
    if (tile >= 0 && tile < num_tiles() && !tile_desc(tile).exact && !k_is_fast(sparse, p.K))
        return launch_one<128, 128, 2, 2, 1, 1, false>(fa, fb, sparse, p, st);
    switch (tile) {
#define FP8_CASE(i, bm, bn, wm, wn, occ, pf) \
    case i: return launch_tile<i>(fa, fb, sparse, p, st);
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
