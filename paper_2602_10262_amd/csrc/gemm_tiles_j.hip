// Instantiates GEMM tiles 28-30 of the tile table (exact sums on the LDS-DMA
// ring: FP8 codes in LDS, decoded to BF16 after the fragment reads).
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(28)
FP8_INSTANTIATE(29)
FP8_INSTANTIATE(30)
}  // namespace fp8k
