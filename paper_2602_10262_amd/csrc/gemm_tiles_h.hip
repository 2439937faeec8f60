// Instantiates GEMM tiles 23, 24, 25, 26 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(23)
FP8_INSTANTIATE(24)
FP8_INSTANTIATE(25)
FP8_INSTANTIATE(26)
}  // namespace fp8k
