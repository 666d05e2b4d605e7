// MFMA tile kernels for bfloat16 operands (grouped launches; one translation unit per
// operand type and launch form so that the library builds in parallel).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch_grouped<OP_BF16>(const GemmArgs *, const int *, int, int, int, int, int, hipStream_t);

}  // namespace psvt
