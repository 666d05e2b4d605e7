// gfx950 (CDNA4) host launchers and the small kernels of the method:
// tile-configuration choice and cost model for the MFMA products (whose
// device code lives in tile.h and is instantiated one operand type and tile
// configuration per unit in gemm_<type>_<tile>.hip), Frobenius norms with
// FP64 accumulation, and the element-wise tile operations (scaling,
// transposition, shifts, conversion to the low-precision operand formats).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "batched.h"
#include "bodies.h"
#include "device.h"
#include "kernels.h"
#include "tilemodel.h"
#include "trace.h"

namespace psvt {

// ------------------------------------------------------------ launching

// Tile configurations: block tile, blocks per CU.
struct TileCfg {
    int bm, occ;
    const char *tag;
};
static const TileCfg kTiles[] = {{0, 0, ""}, {64, 4, "64"}, {128, 2, "128"}, {192, 1, "192"}, {256, 1, "256"}};
static const char *kTypeTag[4] = {"f32", "bf16", "fp8", "bf16x3"};

// Cost model of one product in configuration c (tilemodel.h), with the
// efficiency and per-tile overhead per operand type, kind and configuration
// from the autotuner's table (psvt_tune_set / psvt_tune_load).  Defaults: a
// measured start.
static const float kDefaultEff[4][2][kNumTiles + 1] = {
    {{0.f, 0.78f, 0.86f, 0.73f, 0.76f}, {0.f, 0.64f, 0.72f, 0.72f, 0.45f}},
    {{0.f, 0.30f, 0.40f, 0.40f, 0.45f}, {0.f, 0.30f, 0.40f, 0.40f, 0.45f}},
    {{0.f, 0.25f, 0.35f, 0.35f, 0.40f}, {0.f, 0.25f, 0.35f, 0.35f, 0.40f}},
    {{0.f, 0.40f, 0.45f, 0.40f, 0.45f}, {0.f, 0.40f, 0.45f, 0.40f, 0.45f}},
};
static const float kDefaultOverhead[4][2][kNumTiles + 1] = {
    {{0.f, 19.0f, 51.0f, 17.0f, 0.0f}, {0.f, 14.0f, 20.0f, 15.0f, 19.0f}},
    {{0.f, 6.0f, 8.0f, 10.0f, 12.0f}, {0.f, 6.0f, 8.0f, 10.0f, 12.0f}},
    {{0.f, 6.0f, 8.0f, 10.0f, 12.0f}, {0.f, 6.0f, 8.0f, 10.0f, 12.0f}},
    {{0.f, 8.0f, 10.0f, 12.0f, 14.0f}, {0.f, 8.0f, 10.0f, 12.0f, 14.0f}},
};
static TileModelTable make_default_table() {
    TileModelTable t;
    memcpy(t.eff, kDefaultEff, sizeof t.eff);
    memcpy(t.overhead_us, kDefaultOverhead, sizeof t.overhead_us);
    t.force = 0;
    for (int k = 0; k < 4; ++k) t.max_tile[k] = kNumTiles;
    return t;
}
static TileModelTable g_table = make_default_table();
static thread_local int g_force_tile = 0;
static thread_local int g_persist_tiles = 0;

// The model as the calling thread sees it (its forced configuration and tile
// set included).
TileModelTable tile_model() {
    TileModelTable t = g_table;
    t.force = g_force_tile;
    if (g_persist_tiles)
        for (int k = 0; k < 4; ++k) t.max_tile[k] = kPersistMaxTile[k];
    return t;
}

// The model of the persistent batched executor: its tile set, no forcing.
TileModelTable tile_model_persistent() {
    TileModelTable t = g_table;
    t.force = 0;
    for (int k = 0; k < 4; ++k) t.max_tile[k] = kPersistMaxTile[k];
    return t;
}

static int pick_tile(int type, int M, int N, int K, int sym) { return pick_tile(tile_model(), type, M, N, K, sym); }

template <int ET>
static hipError_t launch_type(const GemmArgs &g, hipStream_t st) {
    const int tile = pick_tile(ET, g.M, g.N, g.K, g.sym);
    const int nblocks = tile_count(g.M, g.N, g.sym, tile_bm(tile));
    if (nblocks == 0) return hipSuccess;
    // useful flops: a symmetric product counts its lower triangle only
    const double flops = g.sym ? (double)g.M * (g.M + 1) * g.K : 2.0 * g.M * g.N * g.K;
    char name[40];
    snprintf(name, sizeof name, "%s_%s_%s", g.sym ? "syrk" : (g.A2 ? "gemm2" : "gemm"), kTypeTag[ET],
             kTiles[tile].tag);
    TraceScope tr(st, trace_name(name), flops, 0.0);
    return gemm_launch<ET>(g, tile, nblocks, st);
}

hipError_t launch_gemm(const GemmArgs &g_in, int op_type, hipStream_t st) {
    if (g_in.M <= 0 || g_in.N <= 0) return hipSuccess;
    if (op_type != OP_F32 && g_in.A2) return hipErrorInvalidValue;
    GemmArgs g = g_in;
    gemm_prepare(g, op_type);
    switch (op_type) {
        case OP_F32: return launch_type<OP_F32>(g, st);
        case OP_BF16: return launch_type<OP_BF16>(g, st);
        case OP_FP8: return launch_type<OP_FP8>(g, st);
        case OP_BF16X3: return launch_type<OP_BF16X3>(g, st);
        default: return hipErrorInvalidValue;
    }
}

void tune_force_tile(int c) { g_force_tile = c; }
void tune_persistent_tiles(int on) { g_persist_tiles = on ? 1 : 0; }
int tune_set_model(int type, int c, int sym, float e, float overhead_us) {
    if (type < 0 || type > 3 || c < 1 || c > kNumTiles || (sym != 0 && sym != 1) || !(e > 0.0f && e <= 1.0f) ||
        !(overhead_us >= 0.0f && overhead_us < 1e6f))
        return -1;
    g_table.eff[type][sym][c] = e;
    g_table.overhead_us[type][sym][c] = overhead_us;
    return 0;
}
int tune_pick(int type, int M, int N, int K, int sym) { return pick_tile(type, M, N, K, sym); }

// ---------------------------------------------------------------- norms

__device__ __forceinline__ int find_group(const int *prefix, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void fro_partial(NormOp op) {
    __shared__ double red[256];
    fro_partial_body(op, blockIdx.x, red);
}
__global__ __launch_bounds__(256) void fro_final(NormOp op) {
    __shared__ double red[256];
    fro_final_body(op, red);
}
__global__ __launch_bounds__(256) void fro_partial_grouped(const NormOp *ops, const int *prefix, int n) {
    __shared__ double red[256];
    const int p = find_group(prefix, n, blockIdx.x);
    const NormOp op = ops[p];  // in registers, not re-read from the table after stores
    fro_partial_body(op, blockIdx.x - prefix[p], red);
}
__global__ __launch_bounds__(256) void fro_final_grouped(const NormOp *ops) {
    __shared__ double red[256];
    const NormOp op = ops[blockIdx.x];
    fro_final_body(op, red);
}

// Batched forms (psvt_svt_batched): a fixed grid loops over the items of
// every matrix (partial sums, or matrices for the final reduction), each
// item's descriptor rebuilt from the stage template and the matrix record.
__global__ __launch_bounds__(256) void fro_partial_batched(BatchView v, NormStageT st) {
    __shared__ double red[256];
    const int total = v.prefix[v.count];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = owner_of(v.prefix, v.count, t);
        const MatInfo mi = v.mats[i];
        NormOp op;
        relocate_norm(st, mi, v.op, v.lp, op);
        fro_partial_body(op, t - v.prefix[i], red);
        __syncthreads();
    }
}
__global__ __launch_bounds__(256) void fro_final_batched(BatchView v, NormStageT st) {
    __shared__ double red[256];
    for (int i = blockIdx.x; i < v.count; i += gridDim.x) {
        const MatInfo mi = v.mats[i];
        if (!mi.valid) continue;
        NormOp op;
        relocate_norm(st, mi, v.op, v.lp, op);
        fro_final_body(op, red);
        __syncthreads();
    }
}

NormOp make_norm_op(const float *X, int64_t rows, int64_t cols, int64_t ld, double *partials, Scalars *sc, int mode,
                    double tau) {
    NormOp op;
    memset(&op, 0, sizeof op);
    op.X = X;
    op.rows = rows;
    op.cols = cols;
    op.ld = ld;
    op.part = partials;
    op.nparts = norm_parts(rows, cols);
    op.sc = sc;
    op.mode = mode;
    op.tau = tau;
    op.safety = 1.0;
    op.scale = 1.0;
    op.status = nullptr;
    op.tol = -1.0;
    return op;
}

hipError_t launch_norm_op(const NormOp &op, hipStream_t st) {
    TraceScope tr(st, "fro_norm", 0.0, 4.0 * op.rows * op.cols);
    hipLaunchKernelGGL(fro_partial, dim3(op.nparts), dim3(256), 0, st, op);
    hipLaunchKernelGGL(fro_final, dim3(1), dim3(256), 0, st, op);
    return hipGetLastError();
}

hipError_t launch_fro_norm(const float *X, int64_t rows, int64_t cols, int64_t ld, double *partials,
                           Scalars *sc, int mode, double tau, hipStream_t st) {
    return launch_norm_op(make_norm_op(X, rows, cols, ld, partials, sc, mode, tau), st);
}

hipError_t launch_norm_grouped(const NormOp *ops, const int *prefix, int n, int total_blocks, double bytes,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    TraceScope tr(st, "fro_norm_grouped", 0.0, bytes);
    hipLaunchKernelGGL(fro_partial_grouped, dim3(total_blocks), dim3(256), 0, st, ops, prefix, n);
    hipLaunchKernelGGL(fro_final_grouped, dim3(n), dim3(256), 0, st, ops);
    return hipGetLastError();
}

// ------------------------------------------------------------- tile ops

__global__ __launch_bounds__(256) void tile_op(TileOp op) {
    __shared__ float lds[64][65];
    tile_op_body(op, blockIdx.x, lds);
}
__global__ __launch_bounds__(256) void tile_op_grouped(const TileOp *ops, const int *prefix, int n) {
    __shared__ float lds[64][65];
    const int p = find_group(prefix, n, blockIdx.x);
    const TileOp op = ops[p];  // in registers, not re-read from the table after stores
    tile_op_body(op, blockIdx.x - prefix[p], lds);
}

__global__ __launch_bounds__(256) void tile_op_batched(BatchView v, TileStageT st) {
    __shared__ float lds[64][65];
    const int total = v.prefix[v.count];
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = owner_of(v.prefix, v.count, t);
        const MatInfo mi = v.mats[i];
        TileOp op;
        relocate_tile(st, mi, v.op, v.lp, op);
        tile_op_body(op, t - v.prefix[i], lds);
        __syncthreads();
    }
}

int tile_op_tiles(const TileOp &op) { return (int)(((op.rows + 63) / 64) * ((op.cols + 63) / 64)); }

double tile_op_bytes(const TileOp &op) {
    const double e = (double)op.rows * op.cols;
    switch (op.kind) {
        case TOP_SCALE_T: return e * 4.0 * (1 + (op.Y != nullptr) + (op.YT != nullptr));
        case TOP_SHIFT: return e * 8.0;
        case TOP_SYMM: return e * 12.0;
        case TOP_WARM: return e * 12.0;
        default: return e * (4.0 + (op.ltype == OP_F32 ? 4 : op.ltype == OP_FP8 ? 1 : op.ltype == OP_BF16 ? 2 : 4));
    }
}

static const char *kTileOpName[5] = {"scale_transpose", "shift_copy", "symmetrize_scale", "convert", "warm_start"};

hipError_t launch_tile_op(const TileOp &op, hipStream_t st) {
    const int n = tile_op_tiles(op);
    if (n <= 0) return hipSuccess;
    TraceScope tr(st, kTileOpName[op.kind], 0.0, tile_op_bytes(op));
    hipLaunchKernelGGL(tile_op, dim3(n), dim3(256), 0, st, op);
    return hipGetLastError();
}

hipError_t launch_tile_op_grouped(const TileOp *ops, const int *prefix, int n, int total, int kind, double bytes,
                                  hipStream_t st) {
    if (n <= 0 || total <= 0) return hipSuccess;
    char name[48];
    snprintf(name, sizeof name, "%s_grouped", kTileOpName[kind]);
    TraceScope tr(st, trace_name(name), 0.0, bytes);
    hipLaunchKernelGGL(tile_op_grouped, dim3(total), dim3(256), 0, st, ops, prefix, n);
    return hipGetLastError();
}

static TileOp blank_op(int kind) {
    TileOp op;
    memset(&op, 0, sizeof op);
    op.kind = kind;
    op.scale = 1.0f;
    op.i_scale = -1;
    return op;
}

TileOp make_scale_transpose(const float *A, int64_t m, int64_t n, int64_t lda, float *Y, int64_t ldy, float *YT,
                            int64_t ldyt, const Scalars *sc, int i_scale) {
    TileOp op = blank_op(TOP_SCALE_T);
    op.X = A;
    op.rows = m;
    op.cols = n;
    op.ldx = lda;
    op.Y = Y;
    op.ldy = ldy;
    op.YT = YT;
    op.ldyt = ldyt;
    op.sc = sc;
    op.i_scale = i_scale;
    return op;
}

TileOp make_shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh, const Scalars *sc,
                       int i_shift) {
    TileOp op = blank_op(TOP_SHIFT);
    op.i_shift = i_shift;
    op.X = T;
    op.rows = op.cols = s;
    op.ldx = ldt;
    op.Y = H;
    op.ldy = ldh;
    op.sc = sc;
    return op;
}

TileOp make_symmetrize_scale(const float *G, int64_t n, int64_t ldg, float *H, int64_t ldh, const Scalars *sc) {
    TileOp op = blank_op(TOP_SYMM);
    op.X = G;
    op.rows = op.cols = n;
    op.ldx = ldg;
    op.Y = H;
    op.ldy = ldh;
    op.sc = sc;
    op.i_scale = F_INV_NU;
    return op;
}

TileOp make_warm_start(const float *H, const float *Z, int64_t ldz, int64_t s, int64_t ldh, float *Y, int64_t ldy,
                       const Scalars *sc, int i_scale, float eps) {
    TileOp op = blank_op(TOP_WARM);
    op.eps = eps;
    op.X = H;
    op.ldx = ldh;
    op.Z = Z;
    op.ldz = ldz;
    op.rows = op.cols = s;
    op.Y = Y;
    op.ldy = ldy;
    op.sc = sc;
    op.i_scale = i_scale;
    return op;
}

TileOp make_convert(const float *X, int64_t rows, int64_t cols, int64_t ld, void *Y, int64_t ldy, int type,
                    float scale, int transpose, const Scalars *sc, int i_scale, int64_t plane) {
    TileOp op = blank_op(TOP_CONVERT);
    op.X = X;
    op.rows = rows;
    op.cols = cols;
    op.ldx = ld;
    op.L = Y;
    op.ldl = ldy;
    op.ltype = type;
    op.ltrans = transpose;
    op.lplane = plane;
    op.scale = scale;
    op.sc = sc;
    op.i_scale = i_scale;
    return op;
}

hipError_t launch_scale_transpose(const float *A, int64_t m, int64_t n, int64_t lda, float *Y, int64_t ldy,
                                  float *YT, int64_t ldyt, const Scalars *sc, int i_scale, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    return launch_tile_op(make_scale_transpose(A, m, n, lda, Y, ldy, YT, ldyt, sc, i_scale), st);
}

hipError_t launch_shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh, const Scalars *sc,
                             hipStream_t st) {
    if (s <= 0) return hipSuccess;
    return launch_tile_op(make_shift_copy(T, s, ldt, H, ldh, sc), st);
}

hipError_t launch_symmetrize_scale(const float *G, int64_t n, int64_t ldg, float *H, int64_t ldh,
                                   const Scalars *sc, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    return launch_tile_op(make_symmetrize_scale(G, n, ldg, H, ldh, sc), st);
}

hipError_t launch_convert(const float *X, int64_t rows, int64_t cols, int64_t ldx, void *Y, int64_t ldy, int type,
                          float scale, int transpose, hipStream_t st, const Scalars *sc, int i_scale, int64_t plane) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    if (type < 0 || type > 3) return hipErrorInvalidValue;
    return launch_tile_op(make_convert(X, rows, cols, ldx, Y, ldy, type, scale, transpose, sc, i_scale, plane), st);
}

// ----------------------------------------------------------- batched forms

hipError_t launch_norm_batched(const BatchView &v, const NormStageT &st, int final_pass, hipStream_t stream) {
    if (final_pass) {
        TraceScope tr(stream, "fro_final_batched", 0.0, 0.0);
        hipLaunchKernelGGL(fro_final_batched, dim3(v.count < 1024 ? (v.count > 0 ? v.count : 1) : 1024), dim3(256), 0,
                           stream, v, st);
    } else {
        TraceScope tr(stream, "fro_partial_batched", 0.0, 0.0);
        hipLaunchKernelGGL(fro_partial_batched, dim3(2048), dim3(256), 0, stream, v, st);
    }
    return hipGetLastError();
}

hipError_t launch_tile_batched(const BatchView &v, const TileStageT &st, hipStream_t stream) {
    char name[48];
    snprintf(name, sizeof name, "%s_batched", kTileOpName[st.t.kind]);
    TraceScope tr(stream, trace_name(name), 0.0, 0.0);
    hipLaunchKernelGGL(tile_op_batched, dim3(2048), dim3(256), 0, stream, v, st);
    return hipGetLastError();
}

hipError_t launch_gemm_batched(const BatchView &v, const GemmStageT &st, int tile, hipStream_t stream) {
    if (st.dtype < OP_F32 || st.dtype > OP_BF16X3 || tile < 1 || tile > kNumTiles) return hipErrorInvalidValue;
    char name[48];
    snprintf(name, sizeof name, "%s_%s_%s_batched", st.g.sym ? "syrk" : (st.r.p[1] ? "gemm2" : "gemm"),
             kTypeTag[st.dtype], kTiles[tile].tag);
    TraceScope tr(stream, trace_name(name), 0.0, 0.0);
    switch (st.dtype) {
        case OP_F32: return gemm_launch_batched<OP_F32>(v, st, tile, stream);
        case OP_BF16: return gemm_launch_batched<OP_BF16>(v, st, tile, stream);
        case OP_FP8: return gemm_launch_batched<OP_FP8>(v, st, tile, stream);
        default: return gemm_launch_batched<OP_BF16X3>(v, st, tile, stream);
    }
}

// ----------------------------------------------------------- grouped GEMM

hipError_t launch_gemm_grouped(const GemmArgs *args, const int *prefix, int n, int total, int op_type, int tile,
                               int sym, int two_a, double flops, hipStream_t st) {
    if (n <= 0 || total <= 0) return hipSuccess;
    if (op_type < OP_F32 || op_type > OP_BF16X3 || tile < 1 || tile > kNumTiles) return hipErrorInvalidValue;
    char name[48];
    snprintf(name, sizeof name, "%s_%s_%s_grouped", sym ? "syrk" : (two_a ? "gemm2" : "gemm"), kTypeTag[op_type],
             kTiles[tile].tag);
    TraceScope tr(st, trace_name(name), flops, 0.0);
    switch (op_type) {
        case OP_F32: return gemm_launch_grouped<OP_F32>(args, prefix, n, total, tile, sym, two_a, st);
        case OP_BF16: return gemm_launch_grouped<OP_BF16>(args, prefix, n, total, tile, sym, two_a, st);
        case OP_FP8: return gemm_launch_grouped<OP_FP8>(args, prefix, n, total, tile, sym, two_a, st);
        default: return gemm_launch_grouped<OP_BF16X3>(args, prefix, n, total, tile, sym, two_a, st);
    }
}

// Host helpers for building grouped launches.
int gemm_pick_tile(const GemmArgs &g, int op_type) { return pick_tile(op_type, g.M, g.N, g.K, g.sym); }
int gemm_tile_count(const GemmArgs &g, int tile) { return tile_count(g.M, g.N, g.sym, tile_bm(tile)); }
double gemm_model_us(const GemmArgs &g, int op_type, int tile) {
    return model_time_us(tile_model(), op_type, g.M, g.N, g.K, g.sym, tile);
}

}  // namespace psvt
