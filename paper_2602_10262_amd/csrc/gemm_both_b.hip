// Both-sides 2:4 kernels of the smaller and exact-sum tiles, and the dispatcher.
#include "gemm_both.hpp"

namespace fp8k {
FP8_BOTH_INSTANTIATE(0)
FP8_BOTH_INSTANTIATE(3)
FP8_BOTH_INSTANTIATE(25)
FP8_BOTH_INSTANTIATE(26)
FP8_BOTH_INSTANTIATE(27)

bool both_tile_supported(int tile)
{
    switch (tile) {
#define FP8_CASE(i) \
    case i: return true;
        FP8_BOTH_TILES(FP8_CASE)
#undef FP8_CASE
    default: return false;
    }
}

hipError_t launch_gemm_both(int tile, int fa, int fb, const GemmParams &p, hipStream_t st)
{
    // K not a multiple of 128: byte-exact loads on the 128 x 128 tile (the
    // exact-sum tiles load byte-exact themselves)
    if (both_tile_supported(tile) && !tile_desc(tile).exact && !k_is_fast(true, p.K))
        return launch_both_one<128, 128, 2, 2, 1, 1, false>(fa, fb, p, st);
    switch (tile) {
#define FP8_CASE(i) \
    case i: return launch_both_tile<i>(fa, fb, p, st);
        FP8_BOTH_TILES(FP8_CASE)
#undef FP8_CASE
    default: return hipErrorInvalidValue;
    }
}
}  // namespace fp8k
