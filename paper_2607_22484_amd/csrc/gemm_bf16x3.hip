// MFMA tile kernels for split-bfloat16 (hi + lo plane) operands (one translation unit per operand type
// so that the library builds in parallel).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch<OP_BF16X3>(const GemmArgs &, int, int, hipStream_t);
template hipError_t gemm_launch_grouped<OP_BF16X3>(const GemmArgs *, const int *, int, int, int, int, int, hipStream_t);

}  // namespace psvt
