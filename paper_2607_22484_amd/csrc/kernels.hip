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

#include <utility>

#include "kernels.h"
#include "trace.h"

namespace psvt {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
// f(0), f(1), ..., f(N-1) with compile-time constant arguments
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

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

// --------------------------------------------------------- operand types

// Storage of one GEMM operand.  Every type moves in 16-byte chunks; an LDS
// row holds 8 chunks (128 bytes) of the k dimension plus a 16-byte pad.
template <int ET>
struct Op;
template <>
struct Op<OP_F32> {
    typedef float T;
    static constexpr int EPC = 4;  // elements per 16-byte chunk
};
template <>
struct Op<OP_BF16> {
    typedef uint16_t T;
    static constexpr int EPC = 8;
};
template <>
struct Op<OP_BF16X3> {
    typedef uint16_t T;
    static constexpr int EPC = 8;
};
template <>
struct Op<OP_FP8> {
    typedef uint8_t T;
    static constexpr int EPC = 16;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

// float -> bfloat16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// float -> OCP FP8 e4m3 (gfx950 hardware conversion, round to nearest even),
// saturated to the largest finite value 448.
__device__ __forceinline__ uint8_t to_fp8(float x) {
    x = fminf(fmaxf(x, -448.0f), 448.0f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false) & 0xFF);
}

// Store one value in a low-precision copy; split bf16 writes hi at idx and
// the residual lo at idx + plane.
__device__ __forceinline__ void store_lp(void *base, int type, int64_t idx, float v, int64_t plane = 0) {
    if (type == OP_BF16) {
        ((uint16_t *)base)[idx] = to_bf16(v);
    } else if (type == OP_BF16X3) {
        const uint16_t hi = to_bf16(v);
        const float hv = __uint_as_float((uint32_t)hi << 16);
        ((uint16_t *)base)[idx] = hi;
        ((uint16_t *)base)[idx + plane] = to_bf16(v - hv);
    } else {
        ((uint8_t *)base)[idx] = to_fp8(v);
    }
}

// One MFMA step pair over 32 bytes of k per lane (two 16-byte chunks).
template <int ET>
__device__ __forceinline__ floatx16 mfma_32b(const u32x4 &a0, const u32x4 &a1, const u32x4 &b0, const u32x4 &b1,
                                             floatx16 acc) {
    if constexpr (ET == OP_F32) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a0[e]), __uint_as_float(b0[e]), acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a1[e]), __uint_as_float(b1[e]), acc, 0, 0, 0);
    } else if constexpr (ET == OP_BF16 || ET == OP_BF16X3) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b0),
                                                      acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1), __builtin_bit_cast(bf16x8, b1),
                                                      acc, 0, 0, 0);
    } else {
        const intx8 a = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
        const intx8 b = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
        // format 0 = FP8 e4m3 for both operands, unit scales (E8M0 127 = 2^0)
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, 127, 0, 127);
    }
    return acc;
}

// Epilogue for one lane's 4 consecutive rows ib..ib+3 of column j:
// v = alpha acc (given) + beta D + diag [i == j], then the FP32 outputs C/CT
// and the low-precision copies Clp/CTlp (value * lp_scale).  SYM: only
// i >= j is kept on diagonal tiles and every kept i != j is also written to
// the mirrored position [j][i].
template <bool SYM>
__device__ __forceinline__ void epilogue_store(const GemmArgs &g, int ib, int j, float v[4], float beta,
                                               bool diag_tile) {
    bool wr[4], mir[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = ib + e;
        if (beta != 0.0f && i < g.M) v[e] += beta * g.D[(int64_t)i * g.ldd + j];
        if (i == j) v[e] += g.diag;
        wr[e] = i < g.M && (!diag_tile || i >= j);
        mir[e] = SYM && wr[e] && i != j;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (!wr[e]) continue;
        const int64_t i = ib + e;
        if (g.C) g.C[i * g.ldc + j] = v[e];
        if (g.Clp) store_lp(g.Clp, g.lp_type, i * g.ldclp + j, v[e] * g.lp_scale, g.lp_plane);
    }
    float *ct = SYM ? g.C : g.CT;
    const int64_t ldct = SYM ? g.ldc : g.ldct;
    const int ctv = SYM ? g.c_vec : g.ct_vec;
    bool t[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) t[e] = SYM ? mir[e] : (ib + e < g.M);
    if (ct) {
        float *p = ct + (int64_t)j * ldct + ib;
        if (ctv && t[0] && t[1] && t[2] && t[3]) {
            *(floatx4 *)p = floatx4{v[0], v[1], v[2], v[3]};
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t[e]) p[e] = v[e];
        }
    }
    void *ctl = SYM ? g.Clp : g.CTlp;
    const int64_t ldctl = SYM ? g.ldclp : g.ldctlp;
    if (ctl) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (t[e]) store_lp(ctl, g.lp_type, (int64_t)j * ldctl + ib + e, v[e] * g.lp_scale, SYM ? g.lp_plane : g.lp_plane_t);
    }
}

// ------------------------------------------------------------------ GEMM

// BM x BN block tile, 256 threads = 2 x 2 waves, each wave (BM/2) x (BN/2)
// made of TM x TN 32x32 MFMA blocks.  A k-tile is 128 bytes of every row
// (32 floats, 64 bf16 or 128 fp8).
//
// MFMA lane layouts (32x32 blocks): lane l feeds row l%32 of A and of B
// (B given as B^T rows) with k-slot group l/32, and holds output
// C[8(r/4) + 4(l/32) + r%4][l%32] in accumulator register r.  The sum over k
// is order-free, so lane half h takes bytes [64h, 64h + 64) of its rows in
// every k-tile: four 16-byte LDS reads per row.  f32 feeds 1 element per
// MFMA (16 MFMAs per k-tile), bf16 8 (4 MFMAs), fp8 32 (2 MFMAs).
template <int ET, int BM, int BN>
struct TileShape {
    static constexpr int ROWB = 144;  // LDS row stride in bytes
    static constexpr int SMEM = 2 * (BM + BN) * ROWB;
};

// Local tile t of a product -> block tile (bi, bj): lower block triangle for
// SYM, grouped row-major order otherwise.
template <bool SYM>
__device__ __forceinline__ void tile_coords(int t, int M, int N, int BM, int BN, int &bi, int &bj) {
    if (SYM)
        tri_index(t, bi, bj);
    else
        grouped_index<8>(t, (M + BM - 1) / BM, (N + BN - 1) / BN, bi, bj);
}

// One BM x BN output tile of the product described by g.
template <int ET, int BM, int BN, bool TWO_A, bool SYM>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int bi, int bj, uint8_t *smem) {
    typedef typename Op<ET>::T T;
    constexpr int EPC = Op<ET>::EPC;
    constexpr int BK = 8 * EPC;        // elements per k-tile
    constexpr int ROWB = TileShape<ET, BM, BN>::ROWB;
    constexpr int TM = BM / 64, TN = BN / 64;
    constexpr int RA = BM / 32, RB = BN / 32;  // 16-byte loads per thread
    const int i0 = bi * BM, j0 = bj * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    const T *A = (const T *)g.A;
    const T *A2 = (const T *)g.A2;
    const T *B = (const T *)g.B;
    float wa = 1.0f, wa2 = 0.0f;
    if constexpr (ET == OP_F32) {
        wa = g.wa * scal(g.sc, g.i_wa);
        wa2 = TWO_A ? g.wa2 * scal(g.sc, g.i_wa2) : 0.0f;
    }

    const int lrow = tid >> 3, lchunk = tid & 7;
    // two register sets: tile k+2 is loaded while tile k is multiplied and
    // tile k+1 waits to be written to LDS (two k-tiles of latency cover)
    // (one set for the largest tiles, where two would not fit in registers)
    constexpr int DEPTH = (BM >= 192) ? 1 : 2;
    u32x4 ra[DEPTH][RA], rb[DEPTH][RB];

    auto load_chunk = [&](const T *P, int64_t ld, int row, int rows, int k) -> u32x4 {
        u32x4 v = {0u, 0u, 0u, 0u};
        if (row < rows) {
            const T *p = P + (int64_t)row * ld + k;
            if (k + EPC <= g.K) {
                v = *(const u32x4 *)p;
            } else {
                // ragged k tail: element-wise, zero beyond K
#pragma unroll
                for (int e = 0; e < EPC; ++e) {
                    uint32_t x = 0u;
                    if (k + e < g.K) {
                        if constexpr (ET == OP_F32)
                            x = __float_as_uint(p[e]);
                        else
                            x = (uint32_t)p[e];
                    }
                    constexpr int SZ = (int)sizeof(T);
                    v[(e * SZ) / 4] |= x << (8 * ((e * SZ) % 4));
                }
            }
        }
        return v;
    };
    // Split bf16: the k loop runs over three virtual segments of Kp = K
    // rounded up to a k-tile; A reads planes (hi, hi, lo), B (hi, lo, hi).
    constexpr bool SPLIT = ET == OP_BF16X3;
    const int Kp = SPLIT ? ((g.K + BK - 1) / BK) * BK : g.K;
    auto gload = [&](int kv, auto set) {
        int k0 = kv, seg = 0;
        if constexpr (SPLIT) {
            seg = kv / Kp;
            k0 = kv - seg * Kp;
        }
        const T *Ap = SPLIT && seg == 2 ? A + g.a_plane : A;
        const T *Bp = SPLIT && seg == 1 ? B + g.b_plane : B;
#pragma unroll
        for (int p = 0; p < RA; ++p) {
            const int r = lrow + 32 * p;
            u32x4 v = load_chunk(Ap, g.lda, i0 + r, g.M, k0 + lchunk * EPC);
            if constexpr (ET == OP_F32) {
                floatx4 f = __builtin_bit_cast(floatx4, v);
                if (TWO_A) {
                    const floatx4 f2 =
                        __builtin_bit_cast(floatx4, load_chunk(A2, g.lda2, i0 + r, g.M, k0 + lchunk * EPC));
                    f = wa * f + wa2 * f2;
                } else {
                    f = wa * f;
                }
                v = __builtin_bit_cast(u32x4, f);
            }
            ra[set][p] = v;
        }
#pragma unroll
        for (int p = 0; p < RB; ++p) rb[set][p] = load_chunk(Bp, g.ldb, j0 + lrow + 32 * p, g.N, k0 + lchunk * EPC);
    };
    auto sstore = [&](int buf, auto set) {
        uint8_t *As = smem + buf * (BM + BN) * ROWB;
        uint8_t *Bs = As + BM * ROWB;
#pragma unroll
        for (int p = 0; p < RA; ++p) *(u32x4 *)&As[(lrow + 32 * p) * ROWB + lchunk * 16] = ra[set][p];
#pragma unroll
        for (int p = 0; p < RB; ++p) *(u32x4 *)&Bs[(lrow + 32 * p) * ROWB + lchunk * 16] = rb[set][p];
    };

    floatx16 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    const int nk = SPLIT ? 3 * (Kp / BK) : (g.K + BK - 1) / BK;
    const int frow = lane & 31, fh = lane >> 5;
    auto compute = [&](int buf) {
        const uint8_t *As = smem + buf * (BM + BN) * ROWB + (wm * (BM / 2)) * ROWB + fh * 64;
        const uint8_t *Bs = smem + buf * (BM + BN) * ROWB + BM * ROWB + (wn * (BN / 2)) * ROWB + fh * 64;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            u32x4 af[TM][2], bf[TN][2];
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                af[a][0] = *(const u32x4 *)&As[(a * 32 + frow) * ROWB + q * 32];
                af[a][1] = *(const u32x4 *)&As[(a * 32 + frow) * ROWB + q * 32 + 16];
            }
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                bf[b][0] = *(const u32x4 *)&Bs[(b * 32 + frow) * ROWB + q * 32];
                bf[b][1] = *(const u32x4 *)&Bs[(b * 32 + frow) * ROWB + q * 32 + 16];
            }
#pragma unroll
            for (int a = 0; a < TM; ++a)
#pragma unroll
                for (int b = 0; b < TN; ++b)
                    acc[a][b] = mfma_32b<ET>(af[a][0], af[a][1], bf[b][0], bf[b][1], acc[a][b]);
        }
    };
    gload(0, std::integral_constant<int, 0>{});
    sstore(0, std::integral_constant<int, 0>{});
    if constexpr (DEPTH == 2) {
        // unrolled by two so that register sets are indexed by constants
        if (nk > 1) gload(BK, std::integral_constant<int, 1>{});
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            if (kt + 2 < nk) gload((kt + 2) * BK, std::integral_constant<int, 0>{});
            compute(0);
            if (kt + 1 < nk) sstore(1, std::integral_constant<int, 1>{});
            __syncthreads();
            if (kt + 1 >= nk) break;
            if (kt + 3 < nk) gload((kt + 3) * BK, std::integral_constant<int, 1>{});
            compute(1);
            if (kt + 2 < nk) sstore(0, std::integral_constant<int, 0>{});
            __syncthreads();
        }
    } else {
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int buf = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * BK, std::integral_constant<int, 0>{});
            compute(buf);
            if (kt + 1 < nk) sstore(buf ^ 1, std::integral_constant<int, 0>{});
            __syncthreads();
        }
    }

    // ------------------------------------------------------------ epilogue
    const float alpha = g.alpha * scal(g.sc, g.i_alpha) * g.ab_scale;
    const float beta = g.D ? g.beta * scal(g.sc, g.i_beta) : 0.0f;
    const bool diag_tile = SYM && (bi == bj);
    // compile-time loops: the accumulator array must only ever be indexed
    // with constants, or it leaves the register file
    static_for<TM>([&](auto a) {
        static_for<TN>([&](auto b) {
            const int j = j0 + wn * (BN / 2) + b * 32 + frow;
            const bool jok = j < g.N;
            static_for<4>([&](auto rg) {
                const int ib = i0 + wm * (BM / 2) + a * 32 + rg * 8 + fh * 4;  // rows ib .. ib+3
                float v[4];
                static_for<4>([&](auto e) { v[e] = alpha * acc[a][b][rg * 4 + e]; });
                if (jok) epilogue_store<SYM>(g, ib, j, v, beta, diag_tile);
            });
        });
    });
}

// One product: block b computes local tile xcd_remap(b) (each XCD gets a
// contiguous range of tiles, so tiles sharing panels share an L2).
template <int ET, int BM, int BN, int OCC, bool TWO_A, bool SYM>
__global__ __launch_bounds__(256, OCC) void gemm_nt(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileShape<ET, BM, BN>::SMEM];
    int bi, bj;
    tile_coords<SYM>(xcd_remap(blockIdx.x, gridDim.x), g.M, g.N, BM, BN, bi, bj);
    gemm_tile<ET, BM, BN, TWO_A, SYM>(g, bi, bj, smem);
}

// Many products of one kind in one launch (batched and serving forms):
// prefix[p] = tiles of products 0..p-1; block b finds its product by binary
// search, so the hardware dispatcher balances uneven products (they are
// ordered largest first).
template <int ET, int BM, int BN, int OCC, bool TWO_A, bool SYM>
__global__ __launch_bounds__(256, OCC) void gemm_grouped(const GemmArgs *args, const int *prefix, int nprob) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileShape<ET, BM, BN>::SMEM];
    const int b = blockIdx.x;
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {  // last p with prefix[p] <= b
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const GemmArgs &g = args[lo];
    int bi, bj;
    tile_coords<SYM>(b - prefix[lo], g.M, g.N, BM, BN, bi, bj);
    gemm_tile<ET, BM, BN, TWO_A, SYM>(g, bi, bj, smem);
}

// ------------------------------------------------------------ launching

// Tile configurations: block tile, blocks per CU.
struct TileCfg {
    int bm, occ;
    const char *tag;
};
static const TileCfg kTiles[] = {{0, 0, ""}, {64, 4, "64"}, {128, 2, "128"}, {192, 1, "192"}, {256, 1, "256"}};
constexpr int kNumTiles = 4;
static const char *kTypeTag[4] = {"f32", "bf16", "fp8", "bf16x3"};
// dense MFMA flop/s of one CU per operand type (257 = 256 CUs + 1)
static const double kCuRate[3] = {157.3e12 / 256.0, 2516.6e12 / 256.0, 5033.2e12 / 256.0};

// Cost model of one product in configuration c:  time ~= (most tiles on one
// CU) x (overhead + tile flops / (efficiency x CU MFMA rate)), with the
// efficiency and per-tile overhead (microseconds) per operand type, kind
// (sym = lower-triangle product) and configuration, from the autotuner's
// table (psvt_tune_set / psvt_tune_load).  Defaults: a measured start.
struct TileModel {
    float eff, overhead_us;
};
static TileModel g_model[3][2][kNumTiles + 1] = {
    {{{0.f, 0.f}, {0.78f, 19.0f}, {0.86f, 51.0f}, {0.73f, 17.0f}, {0.76f, 0.0f}},
     {{0.f, 0.f}, {0.64f, 14.0f}, {0.72f, 20.0f}, {0.72f, 15.0f}, {0.45f, 19.0f}}},
    {{{0.f, 0.f}, {0.30f, 6.0f}, {0.40f, 8.0f}, {0.40f, 10.0f}, {0.45f, 12.0f}},
     {{0.f, 0.f}, {0.30f, 6.0f}, {0.40f, 8.0f}, {0.40f, 10.0f}, {0.45f, 12.0f}}},
    {{{0.f, 0.f}, {0.25f, 6.0f}, {0.35f, 8.0f}, {0.35f, 10.0f}, {0.40f, 12.0f}},
     {{0.f, 0.f}, {0.25f, 6.0f}, {0.35f, 8.0f}, {0.35f, 10.0f}, {0.40f, 12.0f}}},
};
static thread_local int g_force_tile = 0;

static int tile_count(int M, int N, int sym, int bm) {
    const int nbm = (M + bm - 1) / bm, nbn = (N + bm - 1) / bm;
    return sym ? nbm * (nbm + 1) / 2 : nbm * nbn;
}

static double model_time_us(int type, int M, int N, int K, int sym, int c) {
    if (type == OP_BF16X3) {  // three bf16 passes
        type = OP_BF16;
        K *= 3;
    }
    const double bm = kTiles[c].bm;
    const double per_cu = ceil(tile_count(M, N, sym, kTiles[c].bm) / 256.0);
    const TileModel &tm = g_model[type][sym ? 1 : 0][c];
    return per_cu * (tm.overhead_us + 1e6 * bm * bm * 2.0 * K / (tm.eff * kCuRate[type]));
}

static int pick_tile(int type, int M, int N, int K, int sym) {
    if (g_force_tile >= 1 && g_force_tile <= kNumTiles) return g_force_tile;
    double best = 1e300;
    int arg = 2;
    for (int c = 1; c <= kNumTiles; ++c) {
        const double t = model_time_us(type, M, N, K, sym, c);
        if (t < best * 0.999) {
            best = t;
            arg = c;
        }
    }
    return arg;
}

template <int ET, int BM, int OCC>
static hipError_t launch_cfg(const GemmArgs &g, hipStream_t st, const char *tag) {
    const int nblocks = tile_count(g.M, g.N, g.sym, BM);
    if (nblocks == 0) return hipSuccess;
    // useful flops: a symmetric product counts its lower triangle only
    const double flops = g.sym ? (double)g.M * (g.M + 1) * g.K : 2.0 * g.M * g.N * g.K;
    char name[40];
    snprintf(name, sizeof name, "%s_%s_%s", g.sym ? "syrk" : (g.A2 ? "gemm2" : "gemm"), kTypeTag[ET], tag);
    TraceScope tr(st, trace_name(name), flops, 0.0);
    if (g.sym)
        hipLaunchKernelGGL((gemm_nt<ET, BM, BM, OCC, false, true>), dim3(nblocks), dim3(256), 0, st, g);
    else if (ET == OP_F32 && g.A2)
        hipLaunchKernelGGL((gemm_nt<ET, BM, BM, OCC, ET == OP_F32, false>), dim3(nblocks), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((gemm_nt<ET, BM, BM, OCC, false, false>), dim3(nblocks), dim3(256), 0, st, g);
    return hipGetLastError();
}

template <int ET>
static hipError_t launch_type(const GemmArgs &g, hipStream_t st) {
    switch (pick_tile(ET, g.M, g.N, g.K, g.sym)) {
        case 1: return launch_cfg<ET, 64, 4>(g, st, "64");
        case 3: return launch_cfg<ET, 192, 1>(g, st, "192");
        case 4: return launch_cfg<ET, 256, 1>(g, st, "256");
        default: return launch_cfg<ET, 128, 2>(g, st, "128");
    }
}

hipError_t launch_gemm(const GemmArgs &g_in, int op_type, hipStream_t st) {
    if (g_in.M <= 0 || g_in.N <= 0) return hipSuccess;
    GemmArgs g = g_in;
    g.c_vec = g.C && ((uintptr_t)g.C & 15) == 0 && g.ldc % 4 == 0;
    g.ct_vec = g.CT && ((uintptr_t)g.CT & 15) == 0 && g.ldct % 4 == 0;
    if (op_type != OP_F32 && g.A2) return hipErrorInvalidValue;
    switch (op_type) {
        case OP_F32: return launch_type<OP_F32>(g, st);
        case OP_BF16: return launch_type<OP_BF16>(g, st);
        case OP_FP8: return launch_type<OP_FP8>(g, st);
        case OP_BF16X3: return launch_type<OP_BF16X3>(g, st);
        default: return hipErrorInvalidValue;
    }
}

void tune_force_tile(int c) { g_force_tile = c; }
int tune_set_model(int type, int c, int sym, float e, float overhead_us) {
    if (type < 0 || type > 2 || c < 1 || c > kNumTiles || (sym != 0 && sym != 1) || !(e > 0.0f && e <= 1.0f) ||
        !(overhead_us >= 0.0f && overhead_us < 1e6f))
        return -1;
    g_model[type][sym][c] = TileModel{e, overhead_us};
    return 0;
}
int tune_pick(int type, int M, int N, int K, int sym) { return pick_tile(type, M, N, K, sym); }

// ---------------------------------------------------------------- norms

// Partial sums of squares in FP64 of one matrix: chunk b of nb sums rows
// b, b + nb, ...
__device__ __forceinline__ void fro_partial_body(const NormOp &op, int b, double *red) {
    double acc = 0.0;
    for (int64_t r = b; r < op.rows; r += op.nparts) {
        const float *p = op.X + r * op.ld;
        for (int64_t c = threadIdx.x; c < op.cols; c += 256) {
            const double v = (double)p[c];
            acc += v * v;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) op.part[b] = red[0];
}

// Fixed-order final reduction (deterministic), then the derived scalars.
__device__ __forceinline__ void fro_final_body(const NormOp &op, double *red) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < op.nparts; i += 256) acc += op.part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    Scalars *sc = op.sc;
    const double nrm = sqrt(red[0]);
    sc->d[D_NORM] = nrm;
    if (op.mode == NORM_INPUT) {
        sc->d[D_NU] = nrm;
        sc->f[F_NU] = (float)nrm;
        sc->f[F_INV_NU] = nrm > 0.0 ? (float)(1.0 / nrm) : 0.0f;
        sc->d[D_SHIFT] = nrm > 0.0 ? (op.tau / nrm) * (op.tau / nrm) : 0.0;
    } else if (op.mode == NORM_THETA_P || op.mode == NORM_THETA_S) {
        // theta = sqrt(||M||_F) bounds the spectral radius of the iterate:
        // M = X^T X (or H^2) has eigenvalues mu_i >= 0 and
        // ||M||_F = sqrt(sum mu_i^2) >= mu_max = sigma_max^2.
        const double theta = sqrt(nrm);
        const int base = op.mode == NORM_THETA_P ? F_P1 : F_S1;
        const double it = theta > 0.0 ? 1.0 / theta : 0.0;
        sc->f[base] = (float)it;
        sc->f[base + 1] = (float)(it * it);
        sc->f[base + 2] = (float)(it * it * it * it);
    }
}

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
    fro_partial_body(ops[p], blockIdx.x - prefix[p], red);
}
__global__ __launch_bounds__(256) void fro_final_grouped(const NormOp *ops) {
    __shared__ double red[256];
    fro_final_body(ops[blockIdx.x], red);
}

NormOp make_norm_op(const float *X, int64_t rows, int64_t cols, int64_t ld, double *partials, Scalars *sc, int mode,
                    double tau) {
    NormOp op;
    op.X = X;
    op.rows = rows;
    op.cols = cols;
    op.ld = ld;
    op.part = partials;
    op.nparts = (int)(rows < NORM_PARTIALS ? (rows < 1 ? 1 : rows) : NORM_PARTIALS);
    op.sc = sc;
    op.mode = mode;
    op.tau = tau;
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

// 64 x 64 tiles through LDS, 256 threads, 16 elements each.  One kernel for
// every elementwise pass of the method:
//   TOP_SCALE_T  Y = s X, YT = s X^T (either may be NULL)
//   TOP_SHIFT    Y = X - shift I, the diagonal in FP64 (shift from sc)
//   TOP_SYMM     Y = s (X + X^T) / 2
//   TOP_CONVERT  L = lowp(s X) or lowp(s X^T), s = scale [x sc->f[i_scale]]
__device__ __forceinline__ void tile_op_body(const TileOp &op, int tile, float (*lds)[65]) {
    const int ntc = (int)((op.cols + 63) / 64);
    const int64_t r0 = (int64_t)(tile / ntc) * 64, c0 = (int64_t)(tile % ntc) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const float s = op.scale * (op.sc && op.i_scale >= 0 ? op.sc->f[op.i_scale] : 1.0f);
    if (op.kind == TOP_SYMM) {
        for (int k = ty; k < 64; k += 4) {  // mirrored tile X[c0.., r0..]
            const int64_t r = c0 + k, c = r0 + tx;
            lds[k][tx] = (r < op.rows && c < op.cols) ? op.X[r * op.ldx + c] : 0.0f;
        }
        __syncthreads();
        for (int k = ty; k < 64; k += 4) {
            const int64_t r = r0 + k, c = c0 + tx;
            if (r < op.rows && c < op.cols) op.Y[r * op.ldy + c] = 0.5f * s * (op.X[r * op.ldx + c] + lds[tx][k]);
        }
        return;
    }
    const bool need_t = (op.kind == TOP_SCALE_T && op.YT) || (op.kind == TOP_CONVERT && op.ltrans);
    const double shift = op.kind == TOP_SHIFT ? op.sc->d[D_SHIFT] : 0.0;
    for (int k = ty; k < 64; k += 4) {
        const int64_t r = r0 + k, c = c0 + tx;
        const bool in = r < op.rows && c < op.cols;
        float v = in ? op.X[r * op.ldx + c] : 0.0f;
        if (op.kind == TOP_SHIFT) {
            if (in) op.Y[r * op.ldy + c] = (r == c) ? (float)((double)v - shift) : v;
            continue;
        }
        v *= s;
        if (in) {
            if (op.kind == TOP_SCALE_T && op.Y) op.Y[r * op.ldy + c] = v;
            if (op.kind == TOP_CONVERT && !op.ltrans) {
                if (op.ltype == OP_F32)
                    ((float *)op.L)[r * op.ldl + c] = v;
                else
                    store_lp(op.L, op.ltype, r * op.ldl + c, v, op.lplane);
            }
        }
        if (need_t) lds[k][tx] = v;
    }
    if (!need_t) return;
    __syncthreads();
    for (int k = ty; k < 64; k += 4) {
        const int64_t c = c0 + k, r = r0 + tx;  // out[c][r] = X[r][c]
        if (c >= op.cols || r >= op.rows) continue;
        const float v = lds[tx][k];
        if (op.kind == TOP_SCALE_T) {
            op.YT[c * op.ldyt + r] = v;
        } else if (op.ltype == OP_F32) {
            ((float *)op.L)[c * op.ldl + r] = v;
        } else {
            store_lp(op.L, op.ltype, c * op.ldl + r, v, op.lplane);
        }
    }
}

__global__ __launch_bounds__(256) void tile_op(TileOp op) {
    __shared__ float lds[64][65];
    tile_op_body(op, blockIdx.x, lds);
}
__global__ __launch_bounds__(256) void tile_op_grouped(const TileOp *ops, const int *prefix, int n) {
    __shared__ float lds[64][65];
    const int p = find_group(prefix, n, blockIdx.x);
    tile_op_body(ops[p], blockIdx.x - prefix[p], lds);
}

int tile_op_tiles(const TileOp &op) { return (int)(((op.rows + 63) / 64) * ((op.cols + 63) / 64)); }

double tile_op_bytes(const TileOp &op) {
    const double e = (double)op.rows * op.cols;
    switch (op.kind) {
        case TOP_SCALE_T: return e * 4.0 * (1 + (op.Y != nullptr) + (op.YT != nullptr));
        case TOP_SHIFT: return e * 8.0;
        case TOP_SYMM: return e * 12.0;
        default: return e * (4.0 + (op.ltype == OP_F32 ? 4 : op.ltype == OP_FP8 ? 1 : op.ltype == OP_BF16 ? 2 : 4));
    }
}

static const char *kTileOpName[4] = {"scale_transpose", "shift_copy", "symmetrize_scale", "convert"};

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

TileOp make_shift_copy(const float *T, int64_t s, int64_t ldt, float *H, int64_t ldh, const Scalars *sc) {
    TileOp op = blank_op(TOP_SHIFT);
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

// ----------------------------------------------------------- grouped GEMM

template <int ET, int BM, int OCC>
static hipError_t grouped_cfg(const GemmArgs *args, const int *prefix, int n, int total, int sym, int two_a,
                              double flops, hipStream_t st, const char *tag) {
    char name[48];
    snprintf(name, sizeof name, "%s_%s_%s_grouped", sym ? "syrk" : (two_a ? "gemm2" : "gemm"), kTypeTag[ET], tag);
    TraceScope tr(st, trace_name(name), flops, 0.0);
    if (sym)
        hipLaunchKernelGGL((gemm_grouped<ET, BM, BM, OCC, false, true>), dim3(total), dim3(256), 0, st, args, prefix, n);
    else if (two_a && ET == OP_F32)
        hipLaunchKernelGGL((gemm_grouped<ET, BM, BM, OCC, ET == OP_F32, false>), dim3(total), dim3(256), 0, st, args,
                           prefix, n);
    else
        hipLaunchKernelGGL((gemm_grouped<ET, BM, BM, OCC, false, false>), dim3(total), dim3(256), 0, st, args, prefix,
                           n);
    return hipGetLastError();
}

template <int ET>
static hipError_t grouped_type(const GemmArgs *args, const int *prefix, int n, int total, int tile, int sym, int two_a,
                               double flops, hipStream_t st) {
    switch (tile) {
        case 1: return grouped_cfg<ET, 64, 4>(args, prefix, n, total, sym, two_a, flops, st, "64");
        case 3: return grouped_cfg<ET, 192, 1>(args, prefix, n, total, sym, two_a, flops, st, "192");
        case 4: return grouped_cfg<ET, 256, 1>(args, prefix, n, total, sym, two_a, flops, st, "256");
        default: return grouped_cfg<ET, 128, 2>(args, prefix, n, total, sym, two_a, flops, st, "128");
    }
}

hipError_t launch_gemm_grouped(const GemmArgs *args, const int *prefix, int n, int total, int op_type, int tile,
                               int sym, int two_a, double flops, hipStream_t st) {
    if (n <= 0 || total <= 0) return hipSuccess;
    switch (op_type) {
        case OP_F32: return grouped_type<OP_F32>(args, prefix, n, total, tile, sym, two_a, flops, st);
        case OP_BF16: return grouped_type<OP_BF16>(args, prefix, n, total, tile, sym, two_a, flops, st);
        case OP_FP8: return grouped_type<OP_FP8>(args, prefix, n, total, tile, sym, two_a, flops, st);
        case OP_BF16X3: return grouped_type<OP_BF16X3>(args, prefix, n, total, tile, sym, two_a, flops, st);
        default: return hipErrorInvalidValue;
    }
}

// Host helpers for building grouped launches.
int gemm_pick_tile(const GemmArgs &g, int op_type) { return pick_tile(op_type, g.M, g.N, g.K, g.sym); }
int gemm_tile_count(const GemmArgs &g, int tile) { return tile_count(g.M, g.N, g.sym, kTiles[tile].bm); }
double gemm_model_us(const GemmArgs &g, int op_type, int tile) {
    return model_time_us(op_type, g.M, g.N, g.K, g.sym, tile);
}
void gemm_prepare(GemmArgs &g) {
    g.c_vec = g.C && ((uintptr_t)g.C & 15) == 0 && g.ldc % 4 == 0;
    g.ct_vec = g.CT && ((uintptr_t)g.CT & 15) == 0 && g.ldct % 4 == 0;
}

}  // namespace psvt
