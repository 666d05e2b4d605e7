// MFMA tile kernels for FP8 e4m3 operands (single products; one translation unit per
// operand type and launch form so that the library builds in parallel).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch<OP_FP8>(const GemmArgs &, int, int, hipStream_t);

}  // namespace psvt
