// MFMA tile kernels for split-bfloat16 (hi + lo plane) operands, 256x256 tiles (single, grouped and batched launches).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch_bm<OP_BF16X3, 256, 1>(const GemmArgs &, int, hipStream_t);
template hipError_t gemm_grouped_bm<OP_BF16X3, 256, 1>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
template hipError_t gemm_batched_bm<OP_BF16X3, 256, 1>(const BatchView &, const GemmStageT &, int, hipStream_t);

}  // namespace psvt
