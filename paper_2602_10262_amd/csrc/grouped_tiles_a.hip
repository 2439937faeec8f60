// Instantiates the grouped kernels of tiles 19 and 0 (dense and 2:4 lists).
#include "grouped_kernel.hpp"

namespace fp8k {
FP8_GROUPED_INSTANTIATE(19)
FP8_GROUPED_INSTANTIATE(0)
}  // namespace fp8k
