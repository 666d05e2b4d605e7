// MFMA tile kernels for split-bfloat16 (hi + lo plane) operands: the launch
// dispatchers.  The kernels themselves are instantiated one tile
// configuration per translation unit
// (gemm_bf16x3_<tile>.hip) so that the library builds in parallel.
#include "tile.h"

namespace psvt {

extern template hipError_t gemm_launch_bm<OP_BF16X3, 64, tile_occupancy<OP_BF16X3, 64>()>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_BF16X3, 64, tile_occupancy<OP_BF16X3, 64>()>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
extern template hipError_t gemm_launch_bm<OP_BF16X3, 128, tile_occupancy<OP_BF16X3, 128>()>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_BF16X3, 128, tile_occupancy<OP_BF16X3, 128>()>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
extern template hipError_t gemm_launch_bm<OP_BF16X3, 192, 1>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_BF16X3, 192, 1>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);
extern template hipError_t gemm_launch_bm<OP_BF16X3, 256, 1>(const GemmArgs &, int, hipStream_t);
extern template hipError_t gemm_grouped_bm<OP_BF16X3, 256, 1>(const GemmArgs *, const int *, int, int, int, int, hipStream_t);

extern template hipError_t gemm_batched_bm<OP_BF16X3, 64, tile_occupancy<OP_BF16X3, 64>()>(const BatchView &, const GemmStageT &, int, hipStream_t);
extern template hipError_t gemm_batched_bm<OP_BF16X3, 128, tile_occupancy<OP_BF16X3, 128>()>(const BatchView &, const GemmStageT &, int, hipStream_t);
extern template hipError_t gemm_batched_bm<OP_BF16X3, 192, 1>(const BatchView &, const GemmStageT &, int, hipStream_t);
extern template hipError_t gemm_batched_bm<OP_BF16X3, 256, 1>(const BatchView &, const GemmStageT &, int, hipStream_t);

template hipError_t gemm_launch<OP_BF16X3>(const GemmArgs &, int, int, hipStream_t);
template hipError_t gemm_launch_batched<OP_BF16X3>(const BatchView &, const GemmStageT &, int, hipStream_t);
template hipError_t gemm_launch_grouped<OP_BF16X3>(const GemmArgs *, const int *, int, int, int, int, int, hipStream_t);

}  // namespace psvt
