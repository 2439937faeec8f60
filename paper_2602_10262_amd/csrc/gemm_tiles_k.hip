// Instantiates GEMM tile 31 of the tile table (the 256 x 256 LDS-DMA ring
// on the 32 x 32 x 64 FP8 MFMA).
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(31)
}  // namespace fp8k
