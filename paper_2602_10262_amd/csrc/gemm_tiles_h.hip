// Instantiates GEMM tile 23 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(23)
}  // namespace fp8k
