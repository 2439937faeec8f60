// Instantiates the grouped kernels of tiles 23 and 9 (dense and 2:4 lists).
#include "grouped_kernel.hpp"

namespace fp8k {
FP8_GROUPED_INSTANTIATE(23)
FP8_GROUPED_INSTANTIATE(9)
}  // namespace fp8k
