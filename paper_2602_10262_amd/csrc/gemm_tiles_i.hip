// Instantiates GEMM tile 27 of the tile table (the 8-wave exact-sum tile).
#include "gemm_launch.hpp"

namespace fp8k {
FP8_INSTANTIATE(27)
}  // namespace fp8k
