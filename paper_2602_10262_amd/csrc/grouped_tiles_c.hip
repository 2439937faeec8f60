// Instantiates the grouped kernels of tiles 12 and 13 (dense and 2:4 lists).
#include "grouped_kernel.hpp"

namespace fp8k {
FP8_GROUPED_INSTANTIATE(12)
FP8_GROUPED_INSTANTIATE(13)
}  // namespace fp8k
