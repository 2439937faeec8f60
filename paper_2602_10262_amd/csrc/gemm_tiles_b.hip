// Instantiates GEMM tiles 2, 6, 10, 11 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(2)
FP8_INSTANTIATE(6)
FP8_INSTANTIATE(10)
FP8_INSTANTIATE(11)
}  // namespace fp8k
