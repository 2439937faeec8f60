// Instantiates GEMM tiles 20, 21, 22 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(20)
FP8_INSTANTIATE(21)
FP8_INSTANTIATE(22)
}  // namespace fp8k
