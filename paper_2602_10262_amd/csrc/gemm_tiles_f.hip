// Instantiates GEMM tiles 19 of the tile table.
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(19)
}  // namespace fp8k
