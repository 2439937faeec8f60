// Instantiates the grouped kernels of tiles 17, 7 and 26 (dense and 2:4 lists).
#include "grouped_kernel.hpp"

namespace fp8k {
FP8_GROUPED_INSTANTIATE(17)
FP8_GROUPED_INSTANTIATE(7)
FP8_GROUPED_INSTANTIATE(26)
}  // namespace fp8k
