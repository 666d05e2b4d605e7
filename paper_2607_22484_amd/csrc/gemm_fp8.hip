// MFMA tile kernels for FP8 e4m3 operands: the launch dispatchers.  The kernels
// themselves are instantiated one tile configuration per translation unit
// (gemm_fp8_<tile>.hip) so that the library builds in parallel.
#include "tile.h"

namespace psvt {

extern template hipError_t gemm_launch_bm<OP_FP8, 64, tile_occupancy<OP_FP8, 64>()>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_FP8, 64, tile_occupancy<OP_FP8, 64>()>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
extern template hipError_t gemm_launch_bm<OP_FP8, 128, tile_occupancy<OP_FP8, 128>()>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_FP8, 128, tile_occupancy<OP_FP8, 128>()>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
extern template hipError_t gemm_launch_bm<OP_FP8, 192, 1>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_FP8, 192, 1>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
extern template hipError_t gemm_launch_bm<OP_FP8, 256, 1>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_FP8, 256, 1>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);

extern template hipError_t gemm_batched_bm<OP_FP8, 64, tile_occupancy<OP_FP8, 64>()>(const BatchView &, const GemmStageT &, int, hipStream_t);
extern template hipError_t gemm_batched_bm<OP_FP8, 128, tile_occupancy<OP_FP8, 128>()>(const BatchView &, const GemmStageT &, int, hipStream_t);
extern template hipError_t gemm_batched_bm<OP_FP8, 192, 1>(const BatchView &, const GemmStageT &, int, hipStream_t);
extern template hipError_t gemm_batched_bm<OP_FP8, 256, 1>(const BatchView &, const GemmStageT &, int, hipStream_t);

template hipError_t gemm_launch<OP_FP8>(const GemmArgs &, int, int, hipStream_t);
template hipError_t gemm_launch_batched<OP_FP8>(const BatchView &, const GemmStageT &, int, hipStream_t);
template hipError_t gemm_launch_grouped<OP_FP8>(const GemmArgs *, const int *, int, int, int, int, int, hipStream_t);

}  // namespace psvt
