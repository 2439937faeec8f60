// Instantiates GEMM tiles 17, 18 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(17)
FP8_INSTANTIATE(18)
}  // namespace fp8k
