// Instantiates GEMM tiles 12, 13, 14 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(12)
FP8_INSTANTIATE(13)
FP8_INSTANTIATE(14)
}  // namespace fp8k
