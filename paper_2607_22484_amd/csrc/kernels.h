// Internal interface between the host planner (api.hip) and the gfx950
// kernels (kernels.hip).  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tilemodel.h"

namespace psvt {

// Indices into the per-call device scalar block (float part).
enum ScalarIdx {
    F_INV_NU = 0,  // 1 / ||input||_F
    F_NU = 1,      // ||input||_F
    F_P1 = 2,      // 1 / theta_P, theta_P = sqrt(||X0^T X0||_F) >= sigma_max(X0)
    F_P2 = 3,      // 1 / theta_P^2
    F_P4 = 4,      // 1 / theta_P^4
    F_S1 = 5,      // 1 / theta_S, theta_S = sqrt(||H^2||_F) >= |lambda|_max(H)
    F_S2 = 6,
    F_S4 = 7,
    F_TAU_P = 8,   // tau / theta_P (tau in the input's units): the Gram form's weight of N
    F_COUNT = 16
};
// double part
enum DScalarIdx {
    D_NU = 0,     // ||input||_F
    D_SHIFT = 1,  // (tau / nu)^2: the Gram shift in the scaled problem
    D_NORM = 2,   // last norm reduced
    D_CONV = 3,   // RMS deviation ||S^2 - I||_F / sqrt(s) of the final sign iterate
    D_TAU = 4,    // tau / nu: the linear shift of the H-form (P^T X0 - (tau/nu) I)
    D_COUNT = 8
};

struct Scalars {
    double d[D_COUNT];
    float f[F_COUNT];
};

// Element types of the GEMM operands.  OP_BF16X3 ("split bfloat16") stores
// x = hi + lo as two bf16 planes (hi = bf16(x), lo = bf16(x - hi)); a product
// of two split operands is hi.hi + hi.lo + lo.hi (three bf16 MFMA passes,
// about 16 mantissa bits).
enum OpType { OP_F32 = 0, OP_BF16 = 1, OP_FP8 = 2, OP_BF16X3 = 3 };

// One NT product with a fused prologue and epilogue:
//   W[i][k]  = wa * A[i][k] (+ wa2 * A2[i][k])               (prologue)
//   v[i][j]  = alpha * sum_k W[i][k] B[j][k] + beta * D[i][j] + diag*[i==j]
//   C[i][j]  = v,  CT[j][i] = v                              (epilogue)
// Every float multiplier is (host value) x (device scalar f[idx]) when
// idx >= 0.  sym: M == N, only block tiles with bi >= bj run, and each
// lower-triangle value is written to [i][j] and [j][i].
struct GemmArgs {
    const void *A;
    const void *A2;
    const void *B;
    const float *D;
    float *C;
    float *CT;
    void *Clp;   // optional low-precision row-major copy of v (type lp_type)
    void *CTlp;  // optional low-precision transposed copy
    int64_t lda, lda2, ldb, ldd, ldc, ldct, ldclp, ldctlp;
    int M, N, K;
    float alpha, beta, wa, wa2, diag;
    float lp_scale;  // low-precision copies store v * lp_scale
    float ab_scale;  // accumulator multiplier undoing operand scales (1 for f32)
    int i_alpha, i_beta, i_wa, i_wa2;
    const Scalars *sc;
    int sym;
    int c_vec;       // C may take 16-byte stores (aligned, ldc % 4 == 0)
    int direct;      // operand tiles by direct-to-LDS buffer loads (set by gemm_prepare)
    int ct_vec;      // CT may take 16-byte stores
    int lp_type;     // OpType of Clp/CTlp
    int64_t a_plane, b_plane;  // OP_BF16X3 operands: elements from the hi to the lo plane
    int64_t lp_plane, lp_plane_t;  // OP_BF16X3 copies Clp / CTlp: elements from the hi to the lo plane
};

// One Frobenius-norm reduction (FP64) and the scalars derived from it.
struct NormOp {
    const float *X;
    int64_t rows, cols, ld;
    double *part;  // nparts partial sums
    int nparts;
    Scalars *sc;
    int mode;
    double tau;
    double safety;     // NORM_THETA_*: theta is multiplied by it (>= 1)
    double scale;      // NORM_CONV: D_CONV = scale * norm / sqrt(rows)
    uint32_t *status;  // NORM_STATUS: caller's status word (device)
    double tol;        // NORM_STATUS: convergence threshold on D_CONV (< 0: no check)
};

// One 64x64-tiled elementwise pass (see kernels.hip, tile ops).
enum TileOpKind { TOP_SCALE_T = 0, TOP_SHIFT = 1, TOP_SYMM = 2, TOP_CONVERT = 3, TOP_WARM = 4 };
struct TileOp {
    int kind;
    const float *X;
    int64_t rows, cols, ldx;
    float *Y;
    int64_t ldy;
    float *YT;
    int64_t ldyt;
    void *L;
    int64_t ldl;
    int ltype, ltrans;
    int64_t lplane;
    float scale;
    const Scalars *sc;
    int i_scale;
    int i_shift;  // TOP_SHIFT: the FP64 scalar (D_*) subtracted on the diagonal
    const float *Z;  // TOP_WARM: second input (the previous (I + S)/2)
    int64_t ldz;
    float eps;       // TOP_WARM: weight of the previous sign
};

// Launchers (enqueue only).  Return a hipError_t.
hipError_t launch_gemm(const GemmArgs &g, int op_type, hipStream_t st);
hipError_t launch_fro_norm(const float *X, int64_t rows, int64_t cols, int64_t ld, double *partials,
                           Scalars *sc, int mode, double tau, hipStream_t st);
hipError_t launch_scale_transpose(const float *A, int64_t m, int64_t n, int64_t lda, float *Y, int64_t ldy,
                                  float *YT, int64_t ldyt, const Scalars *sc, int i_scale, hipStream_t st);
hipError_t launch_shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh, const Scalars *sc,
                             hipStream_t st);
hipError_t launch_symmetrize_scale(const float *G, int64_t n, int64_t ldg, float *H, int64_t ldh,
                                   const Scalars *sc, hipStream_t st);
// Y = round(scale * [sc->f[i_scale]] * X) in op_type, optionally transposed.
hipError_t launch_convert(const float *X, int64_t rows, int64_t cols, int64_t ld, void *Y, int64_t ldy,
                          int op_type, float scale, int transpose, hipStream_t st, const Scalars *sc = nullptr,
                          int i_scale = -1, int64_t plane = 0);

NormOp make_norm_op(const float *X, int64_t rows, int64_t cols, int64_t ld, double *partials, Scalars *sc, int mode,
                    double tau);
hipError_t launch_norm_op(const NormOp &op, hipStream_t st);
hipError_t launch_norm_grouped(const NormOp *ops, const int *prefix, int n, int total_blocks, double bytes,
                               hipStream_t st);
TileOp make_scale_transpose(const float *A, int64_t m, int64_t n, int64_t lda, float *Y, int64_t ldy, float *YT,
                            int64_t ldyt, const Scalars *sc, int i_scale);
TileOp make_shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh, const Scalars *sc,
                       int i_shift = D_SHIFT);
TileOp make_symmetrize_scale(const float *G, int64_t n, int64_t ldg, float *H, int64_t ldh, const Scalars *sc);
// Warm start of the sign iteration: Y = (X s + eps (2 Z - I)) / (1 + eps)
// with s = sc->f[i_scale] (Z the previous (I + S)/2, X the shifted Gram, s
// its scale 1/theta_S).
TileOp make_warm_start(const float *H, const float *Z, int64_t ldz, int64_t s, int64_t ldh, float *Y, int64_t ldy,
                       const Scalars *sc, int i_scale, float eps);
TileOp make_convert(const float *X, int64_t rows, int64_t cols, int64_t ld, void *Y, int64_t ldy, int type,
                    float scale, int transpose, const Scalars *sc, int i_scale, int64_t plane);
hipError_t launch_tile_op(const TileOp &op, hipStream_t st);
hipError_t launch_tile_op_grouped(const TileOp *ops, const int *prefix, int n, int total, int kind, double bytes,
                                  hipStream_t st);
int tile_op_tiles(const TileOp &op);
double tile_op_bytes(const TileOp &op);
hipError_t launch_gemm_grouped(const GemmArgs *args, const int *prefix, int n, int total, int op_type, int tile,
                               int sym, int two_a, double flops, hipStream_t st);
int gemm_pick_tile(const GemmArgs &g, int op_type);
int gemm_tile_count(const GemmArgs &g, int tile);
double gemm_model_us(const GemmArgs &g, int op_type, int tile);
// Per-product flags set from the operands: vector stores for C / CT, and
// direct-to-LDS operand loads when there is one operand without prescale
// (no A + A2 sum, no FP32 prologue factor), 16-byte aligned rows and planes,
// and every byte offset a tile can form (rows up to M + 255) representable
// in 31 bits (the ragged last k-tile takes masked register loads).
__host__ __device__ inline void gemm_prepare(GemmArgs &g, int op_type) {
    g.c_vec = g.C && ((uintptr_t)g.C & 15) == 0 && g.ldc % 4 == 0;
    g.ct_vec = g.CT && ((uintptr_t)g.CT & 15) == 0 && g.ldct % 4 == 0;
    const int64_t esz = op_type == OP_FP8 ? 1 : (op_type == OP_F32 ? 4 : 2);
    const bool split = op_type == OP_BF16X3;
    const bool prescaled = op_type == OP_F32 && (g.wa != 1.0f || g.i_wa >= 0);
    g.direct = !g.A2 && !prescaled && g.K > 0 && ((uintptr_t)g.A & 15) == 0 && ((uintptr_t)g.B & 15) == 0 &&
               (g.lda * esz) % 16 == 0 && (g.ldb * esz) % 16 == 0 && (g.M + 256) * g.lda * esz < (1LL << 31) &&
               (g.N + 256) * g.ldb * esz < (1LL << 31) &&
               (!split || ((g.a_plane * esz) % 16 == 0 && (g.b_plane * esz) % 16 == 0));
}
// Raw launches of tile configuration `tile` (1..4 = 64/128/192/256) for
// operand type ET (defined in tile.h, instantiated in gemm_<type>.hip); the
// arguments must have gone through gemm_prepare.
template <int ET>
hipError_t gemm_launch(const GemmArgs &g, int tile, int nblocks, hipStream_t st);
template <int ET>
hipError_t gemm_launch_grouped(const GemmArgs *args, const int *prefix, int n, int total, int tile, int sym,
                               int two_a, hipStream_t st);

// modes for launch_fro_norm
enum NormMode {
    NORM_INPUT = 0,    // D_NU, D_SHIFT (needs tau), F_INV_NU, F_NU
    NORM_THETA_P = 1,  // F_P1, F_P2, F_P4 from theta = sqrt(norm)
    NORM_THETA_S = 2,  // F_S1, F_S2, F_S4
    NORM_ONLY = 3,     // D_NORM only
    NORM_CONV = 4,     // D_CONV = scale * norm / sqrt(rows)
    NORM_STATUS = 5    // norm of the output; writes the status word (below)
};

// Bits of the status word (the values of PSVT_STATUS_* in psvt.h).
enum StatusBits { ST_NONFINITE_INPUT = 1, ST_NONFINITE_OUTPUT = 2, ST_NOT_CONVERGED = 4 };

constexpr int NORM_PARTIALS = 1024;
constexpr int64_t NORM_PART_ELEMS = 65536;

// Partial sums of one norm: at most four rows or 64K elements per part
// (whichever gives more parts: short chains of dependent loads per block),
// at most one part per row and NORM_PARTIALS parts.  Every path uses this
// count, so every path sums in the same order.
__host__ __device__ inline int norm_parts(int64_t rows, int64_t cols) {
    int64_t p = (rows * cols + NORM_PART_ELEMS - 1) / NORM_PART_ELEMS;
    const int64_t by_rows = (rows + 3) / 4;
    if (p < by_rows) p = by_rows;
    if (p > rows) p = rows;
    if (p > NORM_PARTIALS) p = NORM_PARTIALS;
    return (int)(p < 1 ? 1 : p);
}

// Device-described batches (batched.h): one launch per stage (products: per
// tile configuration), enqueue only.
struct BatchView;
struct GemmStageT;
struct NormStageT;
struct TileStageT;
hipError_t launch_gemm_batched(const BatchView &v, const GemmStageT &st, int tile, hipStream_t stream);
hipError_t launch_norm_batched(const BatchView &v, const NormStageT &st, int final_pass, hipStream_t stream);
hipError_t launch_tile_batched(const BatchView &v, const TileStageT &st, hipStream_t stream);
template <int ET>
hipError_t gemm_launch_batched(const BatchView &v, const GemmStageT &s, int tile, hipStream_t st);

// The tile cost model as the calling thread sees it (tilemodel.h).
TileModelTable tile_model();
TileModelTable tile_model_persistent();
void tune_persistent_tiles(int on);
void set_persist_spin_limit(long long polls);  // the calling thread's bound on one persistent wait

// Tile-configuration control (autotuner and tests).
void tune_force_tile(int c);
int tune_set_model(int type, int c, int sym, float e, float overhead_us);
int tune_pick(int type, int M, int N, int K, int sym);

}  // namespace psvt
