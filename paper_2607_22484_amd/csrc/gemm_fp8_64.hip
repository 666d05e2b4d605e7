// MFMA tile kernels for FP8 e4m3 operands, 64x64 tiles (single, grouped and batched launches).
#include "tile.h"

namespace psvt {

template hipError_t gemm_launch_bm<OP_FP8, 64, tile_occupancy<OP_FP8, 64>()>(const GemmArgs &, int, hipStream_t);
template hipError_t gemm_grouped_bm<OP_FP8, 64, tile_occupancy<OP_FP8, 64>()>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
template hipError_t gemm_batched_bm<OP_FP8, 64, tile_occupancy<OP_FP8, 64>()>(const BatchView &, const GemmStageT &, int, hipStream_t);

}  // namespace psvt
