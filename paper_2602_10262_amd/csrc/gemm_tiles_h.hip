// Instantiates GEMM tiles 23, 24 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(23)
FP8_INSTANTIATE(24)
}  // namespace fp8k
