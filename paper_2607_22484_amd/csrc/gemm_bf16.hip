// MFMA tile kernels for bfloat16 operands (single products; one translation unit per
// operand type and launch form so that the library builds in parallel).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch<OP_BF16>(const GemmArgs &, int, int, hipStream_t);

}  // namespace psvt
