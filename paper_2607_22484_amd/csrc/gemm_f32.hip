// MFMA tile kernels for FP32 operands (one translation unit per operand type
// so that the library builds in parallel).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch<OP_F32>(const GemmArgs &, int, int, hipStream_t);
template hipError_t gemm_launch_grouped<OP_F32>(const GemmArgs *, const int *, int, int, int, int, int, hipStream_t);

}  // namespace psvt
