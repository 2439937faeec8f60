// Instantiates GEMM tiles 0, 1, 3, 4, 5, 7, 8, 9 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(0)
FP8_INSTANTIATE(1)
FP8_INSTANTIATE(3)
FP8_INSTANTIATE(4)
FP8_INSTANTIATE(5)
FP8_INSTANTIATE(7)
FP8_INSTANTIATE(8)
FP8_INSTANTIATE(9)
}  // namespace fp8k
