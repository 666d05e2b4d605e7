// MFMA tile kernels for split-bfloat16 (hi + lo plane) operands (single products; one translation unit per
// operand type and launch form so that the library builds in parallel).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch<OP_BF16X3>(const GemmArgs &, int, int, hipStream_t);

}  // namespace psvt
