// gfx950 (CDNA4) kernels for polar-decomposition singular value
// soft-thresholding.
//
// The hot path is a chain of dense products (the polar iterations of
// sections 1-2 of the paper, and the fused form of Proposition 1).  They all
// run through one MFMA tile kernel, `gemm_nt`, in "NT" form
//     C[i][j] = sum_k A[i][k] * B[j][k]
// where both operands are row-major with k contiguous.  Every product of the
// method can be put in this form because its right operand is symmetric
// (X^T X, powers of a symmetric matrix, polynomials in it) or because the
// planner keeps a transposed copy of the rectangular iterate.
//
// LDS layout: an operand tile is BM rows of 128 bytes (32 floats) plus a
// 16-byte pad, so that 16-byte LDS reads and writes of 8 consecutive lanes
// cover all banks once.  Global loads are 16 bytes per lane, 8 lanes per row
// (one 128-byte line), staged in registers while the previous tile is being
// multiplied (double-buffered LDS, one barrier per k-tile).
//
// MFMA: v_mfma_f32_32x32x2_f32.  Lane l feeds A[i = l%32][slot l/32] and
// B[slot l/32][j = l%32] and holds C[8(r/4) + 4(l/32) + r%4][l%32] in
// accumulator register r.  The sum over k is order-free, so lane half h
// takes k = 16h + t at step t: each lane then reads 16 consecutive floats of
// its row (four 16-byte LDS reads) per 32-wide k-tile.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "kernels.h"
#include "trace.h"

namespace psvt {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float scal(const Scalars *sc, int idx) { return idx >= 0 ? sc->f[idx] : 1.0f; }

// ---------------------------------------------------------------- tile map

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of tiles so that the tiles sharing operand panels share an L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, local = b >> 3;
    return x * q + (x < r ? x : r) + local;
}

// Lower block triangle, row-major: t -> (bi, bj) with bi >= bj.
__device__ __forceinline__ void tri_index(int t, int &bi, int &bj) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    bi = i;
    bj = t - i * (i + 1) / 2;
}

// Grouped order for a full grid: GROUP block-rows are swept together so a
// B panel is reused GROUP times while it is hot in L2.
template <int GROUP>
__device__ __forceinline__ void grouped_index(int t, int nbm, int nbn, int &bi, int &bj) {
    const int per_group = GROUP * nbn;
    const int g = t / per_group;
    const int first = g * GROUP;
    const int gsize = min(nbm - first, GROUP);
    const int in = t - g * per_group;
    bi = first + in % gsize;
    bj = in / gsize;
}

// ------------------------------------------------------------- FP32 GEMM

// BM x BN block tile, 256 threads = 2 x 2 waves, each wave (BM/2) x (BN/2)
// made of TM x TN 32x32 MFMA blocks.  BK = 32 floats.
template <int BM, int BN, int OCC, bool TWO_A, bool SYM>
__global__ __launch_bounds__(256, OCC) void gemm_nt_f32(GemmArgs g) {
    constexpr int BK = 32;
    constexpr int LDS = BK + 4;  // row stride in floats (144 bytes)
    constexpr int TM = BM / 64, TN = BN / 64;
    constexpr int RA = BM / 32, RB = BN / 32;  // 16-byte loads per thread
    __shared__ __attribute__((aligned(16))) float smem[2 * (BM + BN) * LDS];

    const int nbm = (g.M + BM - 1) / BM, nbn = (g.N + BN - 1) / BN;
    int bi, bj;
    {
        const int t = xcd_remap(blockIdx.x, gridDim.x);
        if (SYM)
            tri_index(t, bi, bj);
        else
            grouped_index<8>(t, nbm, nbn, bi, bj);
    }
    const int i0 = bi * BM, j0 = bj * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    const float *A = (const float *)g.A;
    const float *A2 = (const float *)g.A2;
    const float *B = (const float *)g.B;
    const float wa = g.wa * scal(g.sc, g.i_wa);
    const float wa2 = TWO_A ? g.wa2 * scal(g.sc, g.i_wa2) : 0.0f;

    const int lrow = tid >> 3, lk = (tid & 7) * 4;
    floatx4 ra[RA], rb[RB];

    auto load_row = [&](const float *P, int64_t ld, int row, int rows, int k) -> floatx4 {
        floatx4 v = {0.f, 0.f, 0.f, 0.f};
        if (row < rows) {
            const float *p = P + (int64_t)row * ld + k;
            if (k + 3 < g.K) {
                v = *(const floatx4 *)p;
            } else {
                if (k + 0 < g.K) v.x = p[0];
                if (k + 1 < g.K) v.y = p[1];
                if (k + 2 < g.K) v.z = p[2];
            }
        }
        return v;
    };
    auto gload = [&](int k0) {
#pragma unroll
        for (int p = 0; p < RA; ++p) {
            const int r = lrow + 32 * p;
            floatx4 v = load_row(A, g.lda, i0 + r, g.M, k0 + lk);
            if (TWO_A) {
                floatx4 v2 = load_row(A2, g.lda2, i0 + r, g.M, k0 + lk);
                v = wa * v + wa2 * v2;
            } else {
                v = wa * v;
            }
            ra[p] = v;
        }
#pragma unroll
        for (int p = 0; p < RB; ++p) rb[p] = load_row(B, g.ldb, j0 + lrow + 32 * p, g.N, k0 + lk);
    };
    auto sstore = [&](int buf) {
        float *As = smem + buf * (BM + BN) * LDS;
        float *Bs = As + BM * LDS;
#pragma unroll
        for (int p = 0; p < RA; ++p) *(floatx4 *)&As[(lrow + 32 * p) * LDS + lk] = ra[p];
#pragma unroll
        for (int p = 0; p < RB; ++p) *(floatx4 *)&Bs[(lrow + 32 * p) * LDS + lk] = rb[p];
    };

    floatx16 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    const int nk = (g.K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    const int frow = lane & 31, fh = lane >> 5;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const float *As = smem + buf * (BM + BN) * LDS + (wm * (BM / 2)) * LDS;
        const float *Bs = smem + buf * (BM + BN) * LDS + BM * LDS + (wn * (BN / 2)) * LDS;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            floatx4 af[TM], bf[TN];
#pragma unroll
            for (int a = 0; a < TM; ++a) af[a] = *(const floatx4 *)&As[(a * 32 + frow) * LDS + fh * 16 + q * 4];
#pragma unroll
            for (int b = 0; b < TN; ++b) bf[b] = *(const floatx4 *)&Bs[(b * 32 + frow) * LDS + fh * 16 + q * 4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a][e], bf[b][e], acc[a][b], 0, 0, 0);
        }
        if (kt + 1 < nk) sstore(buf ^ 1);
        __syncthreads();
    }

    // ------------------------------------------------------------ epilogue
    const float alpha = g.alpha * scal(g.sc, g.i_alpha) * g.ab_scale;
    const float beta = g.D ? g.beta * scal(g.sc, g.i_beta) : 0.0f;
    const bool diag_tile = SYM && (bi == bj);
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int j = j0 + wn * (BN / 2) + b * 32 + frow;
#pragma unroll
            for (int rg = 0; rg < 4; ++rg) {
                const int ib = i0 + wm * (BM / 2) + a * 32 + rg * 8 + fh * 4;  // rows ib .. ib+3
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = ib + e;
                    float x = alpha * acc[a][b][rg * 4 + e];
                    if (beta != 0.0f && i < g.M && j < g.N) x += beta * g.D[(int64_t)i * g.ldd + j];
                    if (i == j) x += g.diag;
                    v[e] = x;
                }
                if (j >= g.N) continue;
                if (!SYM) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ib + e < g.M && g.C) g.C[(int64_t)(ib + e) * g.ldc + j] = v[e];
                    if (g.CT) {
                        float *p = g.CT + (int64_t)j * g.ldct + ib;
                        if (g.ct_vec && ib + 3 < g.M) {
                            *(floatx4 *)p = floatx4{v[0], v[1], v[2], v[3]};
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (ib + e < g.M) p[e] = v[e];
                        }
                    }
                } else if (!diag_tile) {
                    // strictly lower tile: every (i, j) has i > j
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ib + e < g.M) g.C[(int64_t)(ib + e) * g.ldc + j] = v[e];
                    float *p = g.C + (int64_t)j * g.ldc + ib;
                    if (g.c_vec && ib + 3 < g.M) {
                        *(floatx4 *)p = floatx4{v[0], v[1], v[2], v[3]};
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (ib + e < g.M) p[e] = v[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int i = ib + e;
                        if (i >= g.M || i < j) continue;
                        g.C[(int64_t)i * g.ldc + j] = v[e];
                        if (i != j) g.C[(int64_t)j * g.ldc + i] = v[e];
                    }
                }
            }
        }
    }
}

// Tile configurations of the FP32 kernel: block tile, blocks per CU.
struct TileCfg {
    int bm, occ;
    const char *tag;
};
static const TileCfg kTiles[] = {{0, 0, ""}, {64, 4, "64"}, {128, 2, "128"}, {192, 1, "192"}, {256, 1, "256"}};
constexpr int kNumTiles = 4;

// Cost model of one product in configuration c (sym = lower-triangle
// product or full one):  time ~= (most tiles on one CU) x (overhead +
// tile flops / (efficiency x CU FP32 MFMA rate)).  The efficiency and the
// per-tile overhead (prologue/epilogue, in microseconds) come from the
// autotuner's table (psvt_tune_set / psvt_tune_load); these defaults are a
// measured starting point.
struct TileModel {
    float eff, overhead_us;
};
static TileModel g_model[2][kNumTiles + 1] = {
    {{0.f, 0.f}, {0.60f, 4.0f}, {0.72f, 6.0f}, {0.71f, 8.0f}, {0.77f, 10.0f}},
    {{0.f, 0.f}, {0.60f, 4.0f}, {0.70f, 6.0f}, {0.71f, 8.0f}, {0.45f, 10.0f}},
};
static thread_local int g_force_tile = 0;
constexpr double kCuRate = 157.3e12 / 256.0;  // FP32 MFMA flop/s of one CU

int tile_count(const GemmArgs &g, int bm) {
    const int nbm = (g.M + bm - 1) / bm, nbn = (g.N + bm - 1) / bm;
    return g.sym ? nbm * (nbm + 1) / 2 : nbm * nbn;
}

double model_time_us(const GemmArgs &g, int c) {
    const double bm = kTiles[c].bm;
    const double per_cu = ceil(tile_count(g, kTiles[c].bm) / 256.0);
    const TileModel &tm = g_model[g.sym ? 1 : 0][c];
    return per_cu * (tm.overhead_us + 1e6 * bm * bm * 2.0 * g.K / (tm.eff * kCuRate));
}

int pick_tile(const GemmArgs &g) {
    if (g_force_tile >= 1 && g_force_tile <= kNumTiles) return g_force_tile;
    double best = 1e300;
    int arg = 2;
    for (int c = 1; c <= kNumTiles; ++c) {
        const double t = model_time_us(g, c);
        if (t < best * 0.999) {
            best = t;
            arg = c;
        }
    }
    return arg;
}

template <int BM, int OCC>
static hipError_t launch_f32(const GemmArgs &g, hipStream_t st, const char *tag) {
    const int nblocks = tile_count(g, BM);
    if (nblocks == 0) return hipSuccess;
    // useful flops: a symmetric product counts its lower triangle only
    const double flops = g.sym ? (double)g.M * (g.M + 1) * g.K : 2.0 * g.M * g.N * g.K;
    char name[32];
    snprintf(name, sizeof name, "%s_f32_%s", g.sym ? "syrk" : (g.A2 ? "gemm2" : "gemm"), tag);
    TraceScope tr(st, trace_name(name), flops, 0.0);
    if (g.sym)
        hipLaunchKernelGGL((gemm_nt_f32<BM, BM, OCC, false, true>), dim3(nblocks), dim3(256), 0, st, g);
    else if (g.A2)
        hipLaunchKernelGGL((gemm_nt_f32<BM, BM, OCC, true, false>), dim3(nblocks), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((gemm_nt_f32<BM, BM, OCC, false, false>), dim3(nblocks), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g_in, int op_type, hipStream_t st) {
    if (g_in.M <= 0 || g_in.N <= 0) return hipSuccess;
    GemmArgs g = g_in;
    g.c_vec = g.C && ((uintptr_t)g.C & 15) == 0 && g.ldc % 4 == 0;
    g.ct_vec = g.CT && ((uintptr_t)g.CT & 15) == 0 && g.ldct % 4 == 0;
    if (op_type != OP_F32) return hipErrorInvalidValue;
    switch (pick_tile(g)) {
        case 1: return launch_f32<64, 4>(g, st, "64");
        case 3: return launch_f32<192, 1>(g, st, "192");
        case 4: return launch_f32<256, 1>(g, st, "256");
        default: return launch_f32<128, 2>(g, st, "128");
    }
}

void tune_force_tile(int c) { g_force_tile = c; }
int tune_set_model(int c, int sym, float e, float overhead_us) {
    if (c < 1 || c > kNumTiles || (sym != 0 && sym != 1) || !(e > 0.0f && e <= 1.0f) ||
        !(overhead_us >= 0.0f && overhead_us < 1e6f))
        return -1;
    g_model[sym][c] = TileModel{e, overhead_us};
    return 0;
}
int tune_pick(int M, int N, int K, int sym) {
    GemmArgs g;
    memset(&g, 0, sizeof g);
    g.M = M;
    g.N = N;
    g.K = K;
    g.sym = sym;
    return pick_tile(g);
}

// ---------------------------------------------------------------- norms

// Partial sums of squares in FP64: block b sums rows b, b + G, ... .
__global__ __launch_bounds__(256) void fro_partial(const float *X, int64_t rows, int64_t cols, int64_t ld,
                                                   double *part) {
    double acc = 0.0;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const float *p = X + r * ld;
        for (int64_t c = threadIdx.x; c < cols; c += 256) {
            const double v = (double)p[c];
            acc += v * v;
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Fixed-order final reduction, then the derived scalars of `mode`.
__global__ __launch_bounds__(256) void fro_final(const double *part, int nparts, Scalars *sc, int mode,
                                                 double tau) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double nrm = sqrt(red[0]);
    sc->d[D_NORM] = nrm;
    if (mode == NORM_INPUT) {
        sc->d[D_NU] = nrm;
        sc->f[F_NU] = (float)nrm;
        sc->f[F_INV_NU] = nrm > 0.0 ? (float)(1.0 / nrm) : 0.0f;
        sc->d[D_SHIFT] = nrm > 0.0 ? (tau / nrm) * (tau / nrm) : 0.0;
    } else if (mode == NORM_THETA_P || mode == NORM_THETA_S) {
        // theta = sqrt(||M||_F) bounds the spectral radius of the iterate:
        // M = X^T X (or H^2) has eigenvalues mu_i >= 0 and
        // ||M||_F = sqrt(sum mu_i^2) >= mu_max = sigma_max^2.
        const double theta = sqrt(nrm);
        const int base = mode == NORM_THETA_P ? F_P1 : F_S1;
        const double it = theta > 0.0 ? 1.0 / theta : 0.0;
        sc->f[base] = (float)it;
        sc->f[base + 1] = (float)(it * it);
        sc->f[base + 2] = (float)(it * it * it * it);
    }
}

hipError_t launch_fro_norm(const float *X, int64_t rows, int64_t cols, int64_t ld, double *partials,
                           Scalars *sc, int mode, double tau, hipStream_t st) {
    int nb = (int)(rows < NORM_PARTIALS ? rows : NORM_PARTIALS);
    if (nb < 1) nb = 1;
    TraceScope tr(st, "fro_norm", 0.0, 4.0 * rows * cols);
    hipLaunchKernelGGL(fro_partial, dim3(nb), dim3(256), 0, st, X, rows, cols, ld, partials);
    hipLaunchKernelGGL(fro_final, dim3(1), dim3(256), 0, st, partials, nb, sc, mode, tau);
    return hipGetLastError();
}

// ---------------------------------------------------- transpose and copies

// Y = s A (m x n) and YT = s A^T (n x m); either output may be NULL.
// 64 x 64 tiles through LDS, 256 threads, 16 elements each.
__global__ __launch_bounds__(256) void scale_transpose(const float *A, int64_t m, int64_t n, int64_t lda,
                                                       float *Y, int64_t ldy, float *YT, int64_t ldyt,
                                                       const Scalars *sc, int i_scale) {
    __shared__ float tile[64][65];
    const float s = scal(sc, i_scale);
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int k = ty; k < 64; k += 4) {
        const int64_t r = r0 + k, c = c0 + tx;
        float v = 0.0f;
        if (r < m && c < n) {
            v = s * A[r * lda + c];
            if (Y) Y[r * ldy + c] = v;
        }
        tile[k][tx] = v;
    }
    if (!YT) return;
    __syncthreads();
    for (int k = ty; k < 64; k += 4) {
        const int64_t c = c0 + k, r = r0 + tx;  // YT[c][r] = tile[r - r0][c - c0]
        if (c < n && r < m) YT[c * ldyt + r] = tile[tx][k];
    }
}

hipError_t launch_scale_transpose(const float *A, int64_t m, int64_t n, int64_t lda, float *Y, int64_t ldy,
                                  float *YT, int64_t ldyt, const Scalars *sc, int i_scale, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
    TraceScope tr(st, "scale_transpose", 0.0, 4.0 * m * n * (1 + (Y != nullptr) + (YT != nullptr)));
    hipLaunchKernelGGL(scale_transpose, grid, dim3(256), 0, st, A, m, n, lda, Y, ldy, YT, ldyt, sc, i_scale);
    return hipGetLastError();
}

// H = T - shift I with the diagonal subtraction done in FP64
// (shift = (tau/nu)^2 from the scalar block).
__global__ __launch_bounds__(256) void shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh,
                                                  const Scalars *sc) {
    const double shift = sc->d[D_SHIFT];
    for (int64_t r = blockIdx.x; r < s; r += gridDim.x) {
        const float *src = T + r * ldt;
        float *dst = H + r * ldh;
        for (int64_t c = threadIdx.x; c < s; c += 256) {
            float v = src[c];
            if (c == r) v = (float)((double)v - shift);
            dst[c] = v;
        }
    }
}

hipError_t launch_shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh, const Scalars *sc,
                             hipStream_t st) {
    if (s <= 0) return hipSuccess;
    const int nb = (int)(s < 2048 ? s : 2048);
    TraceScope tr(st, "shift_copy", 0.0, 8.0 * s * s);
    hipLaunchKernelGGL(shift_copy, dim3(nb), dim3(256), 0, st, T, s, ldt, H, ldh, sc);
    return hipGetLastError();
}

// H = (G + G^T) / (2 nu), nu = ||G||_F from the scalar block.
__global__ __launch_bounds__(256) void symmetrize_scale(const float *G, int64_t n, int64_t ldg, float *H,
                                                        int64_t ldh, const Scalars *sc) {
    __shared__ float tile[64][65];
    const float s = 0.5f * sc->f[F_INV_NU];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // load the mirrored tile G[c0.., r0..]
    for (int k = ty; k < 64; k += 4) {
        const int64_t r = c0 + k, c = r0 + tx;
        tile[k][tx] = (r < n && c < n) ? G[r * ldg + c] : 0.0f;
    }
    __syncthreads();
    for (int k = ty; k < 64; k += 4) {
        const int64_t r = r0 + k, c = c0 + tx;
        if (r < n && c < n) H[r * ldh + c] = s * (G[r * ldg + c] + tile[tx][k]);
    }
}

hipError_t launch_symmetrize_scale(const float *G, int64_t n, int64_t ldg, float *H, int64_t ldh,
                                   const Scalars *sc, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 63) / 64));
    TraceScope tr(st, "symmetrize_scale", 0.0, 12.0 * n * n);
    hipLaunchKernelGGL(symmetrize_scale, grid, dim3(256), 0, st, G, n, ldg, H, ldh, sc);
    return hipGetLastError();
}

hipError_t launch_convert(const float *, int64_t, int64_t, int64_t, void *, int64_t, int, float, int,
                          hipStream_t) {
    return hipErrorInvalidValue;  // low-precision copies: not built yet
}

}  // namespace psvt
