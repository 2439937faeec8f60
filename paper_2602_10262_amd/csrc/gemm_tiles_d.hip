// Instantiates GEMM tiles 15, 16 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(15)
FP8_INSTANTIATE(16)
}  // namespace fp8k
