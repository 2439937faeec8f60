// Both-sides 2:4 kernels of the 256-row tiles (compiled apart for build parallelism).
#include "gemm_both.hpp"

namespace fp8k {
FP8_BOTH_INSTANTIATE(11)
FP8_BOTH_INSTANTIATE(12)
}  // namespace fp8k
