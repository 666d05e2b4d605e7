// Device code of the MFMA tile kernel shared by every product of the method
// (included by the units gemm_<type>_<tile>.hip, which instantiate one
// operand type and tile configuration each, and gemm_<type>.hip, which
// instantiate the dispatchers).
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
// Two tile bodies share the MFMA schedule and the epilogue:
//  * gemm_tile_direct (whole k-tiles, aligned operands): buffer loads write
//    straight into an unpadded, XOR-swizzled LDS tile;
//  * gemm_tile (everything else: ragged k, the two-operand sum A + A2):
//    16-byte loads staged in registers, LDS rows of 128 bytes plus a 16-byte
//    pad so that 16-byte accesses of 8 consecutive lanes cover all banks once.
//
// MFMA: v_mfma_f32_32x32x2_f32 / 32x32x16_bf16 / scaled 32x32x64 f8f6f4.
// Lane l feeds A[i = l%32] and B[j = l%32] with k-slot group l/32 and holds
// C[8(r/4) + 4(l/32) + r%4][l%32] in accumulator register r.  The sum over k
// is order-free, so lane half h takes bytes [64h, 64h + 64) of its rows in
// every 128-byte k-tile.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <utility>

#include "batched.h"
#include "device.h"
#include "kernels.h"

namespace psvt {

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

// ------------------------------------------------------------- epilogue
// Tiles up to 128 x 128: from the accumulator registers.
// Epilogue for one lane's 4 consecutive rows ib..ib+3 of column j:
// v = alpha acc + beta D (given) + diag [i == j], then the FP32 outputs C/CT
// and the low-precision copies Clp/CTlp (value * lp_scale).  SYM: only
// i >= j is kept on diagonal tiles and every kept i != j is also written to
// the mirrored position [j][i].
template <bool SYM>
__device__ __forceinline__ void epilogue_store(const GemmArgs &g, int ib, int j, float v[4], bool diag_tile) {
    bool wr[4], mir[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = ib + e;
        if (i == j) v[e] += g.diag;
        wr[e] = i < g.M && (!diag_tile || i >= j);
        mir[e] = SYM && wr[e] && i != j;
    }
    if (g.C) {
        float *p = g.C + (int64_t)ib * g.ldc + j;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (wr[e]) p[(int64_t)e * g.ldc] = v[e];
    }
    if (g.Clp) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (wr[e]) store_lp(g.Clp, g.lp_type, (int64_t)(ib + e) * g.ldclp + j, v[e] * g.lp_scale, g.lp_plane);
    }
    float *ct = SYM ? g.C : g.CT;
    const int64_t ldct = SYM ? g.ldc : g.ldct;
    const int ctv = SYM ? g.c_vec : g.ct_vec;
    bool t[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) t[e] = SYM ? mir[e] : (ib + e < g.M);
    const bool all = t[0] && t[1] && t[2] && t[3];
    if (ct) {
        float *p = ct + (int64_t)j * ldct + ib;
        if (ctv && all) {
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
        const int64_t plane = SYM ? g.lp_plane : g.lp_plane_t;
        if (all) {
            store_lp4(ctl, g.lp_type, (int64_t)j * ldctl + ib, v, g.lp_scale, plane);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (t[e]) store_lp(ctl, g.lp_type, (int64_t)j * ldctl + ib + e, v[e] * g.lp_scale, plane);
        }
    }
}

// Scaled accumulators of one block tile -> outputs, one 32-row group of
// the wave's rows at a time.  HAS_D: the D values of row group a + 1 are
// loaded before the stores of group a, so that waiting for them never waits
// for those stores (vector memory counters retire in issue order); without
// D there is no load and no wait between the stores.  Compile-time loops:
// the accumulator array must only ever be indexed with constants, or it
// leaves the register file.
template <int BM, int BN, bool SYM, bool HAS_D>
__device__ __forceinline__ void store_tile_regs_v(const GemmArgs &g, int bi, int bj,
                                                  floatx16 (&acc)[BM / 64][BN / 64], float alpha, float beta,
                                                  const int tid) {
    constexpr int TM = BM / 64, TN = BN / 64;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1, frow = lane & 31, fh = lane >> 5;
    const int i0 = bi * BM + wm * (BM / 2), j0 = bj * BN + wn * (BN / 2) + frow;
    const bool diag_tile = SYM && (bi == bj);
    float dv[HAS_D ? 2 : 1][TN][16];
    auto load_d = [&](auto a) {
        static_for<4>([&](auto rg) {
            const int ib = i0 + a * 32 + rg * 8 + fh * 4;
            const float *drow = g.D + (int64_t)ib * g.ldd + j0;
            static_for<TN>([&](auto b) {
                const int j = j0 + b * 32;
                static_for<4>([&](auto e) {
                    dv[a & 1][b][rg * 4 + e] =
                        (ib + e < g.M && j < g.N) ? drow[(int64_t)e * g.ldd + b * 32] : 0.0f;
                });
            });
        });
    };
    if constexpr (HAS_D) load_d(std::integral_constant<int, 0>{});
    static_for<TM>([&](auto a) {
        if constexpr (HAS_D && a + 1 < TM) load_d(std::integral_constant<int, a + 1>{});
        static_for<TN>([&](auto b) {
            const int j = j0 + b * 32;
            const bool jok = j < g.N;
            static_for<4>([&](auto rg) {
                const int ib = i0 + a * 32 + rg * 8 + fh * 4;  // rows ib .. ib+3
                float v[4];
                static_for<4>([&](auto e) {
                    v[e] = alpha * acc[a][b][rg * 4 + e];
                    if constexpr (HAS_D) v[e] += beta * dv[HAS_D ? (a & 1) : 0][b][rg * 4 + e];
                });
                if (jok) epilogue_store<SYM>(g, ib, j, v, diag_tile);
            });
        });
    });
}

// Tiles of 192 and 256: through LDS.

// The block's accumulators go through LDS (the operand tiles are no longer
// needed) and leave in two passes of short loops over 4-element groups:
//  1. rows: v = alpha acc + beta D + diag [i == j] for 4 consecutive
//     columns of a row; C and the low-precision copy Clp (row-major), and v
//     back into LDS;
//  2. columns (only for CT / CTlp, or the mirrored half of a symmetric
//     product): v of 4 consecutive rows of a column, written to row j of the
//     transposed output.
// SYM: on diagonal tiles only i >= j is kept, and every kept i != j is also
// written to [j][i].  The values and every output element are those of a
// lane-by-lane epilogue; the loops keep the code compact (a fully unrolled
// epilogue of a 256 x 256 tile is several hundred KB of instructions).
// Tiles of 192 and 256 rows are staged in two halves of rows.
// LDS layout: element (r, c) of a chunk at r * BN + (c ^ swz(r)), swz(r) =
// 8 ((r / 4) mod 8).  The XOR moves 8-column groups within their 64-column
// block, so 4-column groups stay contiguous and 16-byte aligned, and:
//  * a 16-lane phase of pass 1 (16 consecutive 4-column groups of a row)
//    reads one 64-float block, all banks once;
//  * pass 2 gives a wave 32 rows x 8 columns: lane (li, lj) holds rows
//    4 li .. 4 li + 3 of column 8 cg + lj, at bank 8 (cg ^ li) + lj (all
//    64 banks once per row offset), and the 8 lanes of one column write 128
//    contiguous bytes of the transposed row.
template <int BM, int BN>
struct EpiShape {
    static constexpr int NCH = BM >= 192 ? 2 : 1;  // row chunks
    static constexpr int RC = BM / NCH;            // rows per chunk
    static constexpr int BYTES = RC * BN * 4;
    static_assert(BN % 64 == 0 && RC % 32 == 0, "whole 64-column blocks, 32-row groups");
    // the register-staged body's LDS (the smallest of any operand type)
    static_assert(BYTES <= 2 * (BM + BN) * 144, "epilogue staging fits the tile's LDS");
};
__device__ __forceinline__ int epi_idx(int r, int c, int bn) { return r * bn + (c ^ (((r >> 2) & 7) << 3)); }

template <int BM, int BN, bool SYM>
__device__ __forceinline__ void store_tile_lds(const GemmArgs &g, int bi, int bj, floatx16 (&acc)[BM / 64][BN / 64],
                                               uint8_t *smem, const int tid) {
    static_assert(BM == BN, "square block tiles");
    typedef EpiShape<BM, BN> E;
    constexpr int TPR = BN / 4;  // 4-column groups per row
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1, frow = lane & 31, fh = lane >> 5;
    const int i0 = bi * BM, j0 = bj * BN;
    const float alpha = g.alpha * scal(g.sc, g.i_alpha) * g.ab_scale;
    const float beta = g.D ? g.beta * scal(g.sc, g.i_beta) : 0.0f;
    const bool diag_tile = SYM && (bi == bj);
    const bool d_vec = ((uintptr_t)g.D & 15) == 0 && g.ldd % 4 == 0;
    // the transposed outputs: CT / CTlp, or the mirror of a symmetric product
    float *tc = SYM ? g.C : g.CT;
    void *tl = SYM ? g.Clp : g.CTlp;
    const int64_t ldtc = SYM ? g.ldc : g.ldct, ldtl = SYM ? g.ldclp : g.ldctlp;
    const int64_t tplane = SYM ? g.lp_plane : g.lp_plane_t;
    const bool tvec = SYM ? g.c_vec : g.ct_vec;
    float *L = (float *)smem;
    static_for<E::NCH>([&](auto c) {
        const int r0 = c * E::RC;  // first tile row of this chunk
        __syncthreads();           // LDS free: operand tiles (or the previous chunk) consumed
        if (E::NCH == 1 || wm == c) {
            static_for<BM / 64>([&](auto a) {
                static_for<BN / 64>([&](auto b) {
                    static_for<16>([&](auto r) {
                        const int row = wm * (BM / 2) + a * 32 + (r / 4) * 8 + fh * 4 + (r % 4) - r0;
                        const int col = wn * (BN / 2) + b * 32 + frow;
                        L[epi_idx(row, col, BN)] = acc[a][b][(int)r];
                    });
                });
            });
        }
        __syncthreads();
        // pass 1: rows
        for (int q = tid; q < E::RC * TPR; q += 256) {
            const int lr = q / TPR, lc = (q - lr * TPR) * 4;
            const int i = i0 + r0 + lr, j = j0 + lc;
            floatx4 *lp = (floatx4 *)&L[epi_idx(lr, lc, BN)];
            const floatx4 a4 = *lp;
            float v[4];
            bool ok[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ok[e] = i < g.M && j + e < g.N && (!diag_tile || i >= j + e);
                v[e] = alpha * a4[e];
            }
            if (beta != 0.0f) {
                const float *dp = g.D + (int64_t)i * g.ldd + j;
                if (d_vec && i < g.M && j + 3 < g.N) {
                    const floatx4 d4 = *(const floatx4 *)dp;
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] += beta * d4[e];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] += beta * ((i < g.M && j + e < g.N) ? dp[e] : 0.0f);
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i == j + e) v[e] += g.diag;
            const bool all = ok[0] && ok[1] && ok[2] && ok[3];
            if (g.C) {
                float *cp = g.C + (int64_t)i * g.ldc + j;
                if (all && g.c_vec) {
                    *(floatx4 *)cp = floatx4{v[0], v[1], v[2], v[3]};
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ok[e]) cp[e] = v[e];
                }
            }
            if (g.Clp) {
                if (all) {
                    store_lp4(g.Clp, g.lp_type, (int64_t)i * g.ldclp + j, v, g.lp_scale, g.lp_plane);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (ok[e]) store_lp(g.Clp, g.lp_type, (int64_t)i * g.ldclp + j + e, v[e] * g.lp_scale, g.lp_plane);
                }
            }
            *lp = floatx4{v[0], v[1], v[2], v[3]};
        }
        if (tc || tl) {
            __syncthreads();
            // pass 2: columns (4 consecutive rows of column j -> row j of
            // the transposed output); each wave takes 32 rows x 8 columns
            for (int q = tid; q < E::RC * BN / 4; q += 256) {
                const int lj = q & 7, li = (q >> 3) & 7, blk = q >> 6;
                const int rb = blk / (BN / 8), cg = blk - rb * (BN / 8);
                const int lr = rb * 32 + li * 4, lc = cg * 8 + lj;
                const int i = i0 + r0 + lr, j = j0 + lc;
                float v[4];
                bool ok[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = L[epi_idx(lr + e, lc, BN)];
                    ok[e] = i + e < g.M && j < g.N && (!SYM || !diag_tile || i + e > j);
                }
                const bool all = ok[0] && ok[1] && ok[2] && ok[3];
                if (tc) {
                    float *p = tc + (int64_t)j * ldtc + i;
                    if (all && tvec) {
                        *(floatx4 *)p = floatx4{v[0], v[1], v[2], v[3]};
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (ok[e]) p[e] = v[e];
                    }
                }
                if (tl) {
                    if (all) {
                        store_lp4(tl, g.lp_type, (int64_t)j * ldtl + i, v, g.lp_scale, tplane);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (ok[e]) store_lp(tl, g.lp_type, (int64_t)j * ldtl + i + e, v[e] * g.lp_scale, tplane);
                    }
                }
            }
        }
    });
}

// One epilogue per block tile.  Up to 128 x 128 the per-lane epilogue is
// a few KB of code; the 192/256 tiles leave through LDS, whose loops keep
// the kernel within the instruction cache.
template <int BM, int BN, bool SYM>
__device__ __forceinline__ void store_tile(const GemmArgs &g, int bi, int bj, floatx16 (&acc)[BM / 64][BN / 64],
                                           uint8_t *smem, const int tid = (int)threadIdx.x) {
    if constexpr (BM >= 192) {
        store_tile_lds<BM, BN, SYM>(g, bi, bj, acc, smem, tid);
    } else {
        static_assert(BM == BN, "square block tiles");
        const float alpha = g.alpha * scal(g.sc, g.i_alpha) * g.ab_scale;
        const float beta = g.D ? g.beta * scal(g.sc, g.i_beta) : 0.0f;
        if (beta != 0.0f)
            store_tile_regs_v<BM, BN, SYM, true>(g, bi, bj, acc, alpha, beta, tid);
        else
            store_tile_regs_v<BM, BN, SYM, false>(g, bi, bj, acc, alpha, beta, tid);
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
    static constexpr int ROWB = 144;  // LDS row stride in bytes (register-staged body)
    // split bf16 up to 128 x 128: the direct body keeps both planes per stage
    static constexpr bool FUSED_SPLIT = ET == OP_BF16X3 && BM <= 128 && BN <= 128;
    static constexpr int STAGED = 2 * (BM + BN) * ROWB;
    static constexpr int DIRECT = (FUSED_SPLIT ? 4 : 2) * (BM + BN) * 128;
    static constexpr int SMEM = STAGED > DIRECT ? STAGED : DIRECT;
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

// One 16-byte chunk of row `row` starting at element k: zero for rows past
// `rows`; element-wise with zeros beyond K on a ragged k tail.
template <int ET>
__device__ __forceinline__ u32x4 load_chunk_masked(const typename Op<ET>::T *P, int64_t ld, int row, int rows, int k,
                                                   int K) {
    typedef typename Op<ET>::T T;
    constexpr int EPC = Op<ET>::EPC;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (row < rows) {
        const T *p = P + (int64_t)row * ld + k;
        if (k + EPC <= K) {
            v = *(const u32x4 *)p;
        } else {
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                uint32_t x = 0u;
                if (k + e < K) {
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
}

// One BM x BN output tile of the product described by g.
template <int ET, int BM, int BN, bool TWO_A, bool SYM>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int bi, int bj, uint8_t *smem,
                                          floatx16 (&acc)[BM / 64][BN / 64], const int tid = (int)threadIdx.x) {
    typedef typename Op<ET>::T T;
    constexpr int EPC = Op<ET>::EPC;
    constexpr int BK = 8 * EPC;        // elements per k-tile
    constexpr int ROWB = TileShape<ET, BM, BN>::ROWB;
    constexpr int TM = BM / 64, TN = BN / 64;
    constexpr int RA = BM / 32, RB = BN / 32;  // 16-byte loads per thread
    const int i0 = bi * BM, j0 = bj * BN;
    const int lane = tid & 63, wave = tid >> 6;
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
        return load_chunk_masked<ET>(P, ld, row, rows, k, g.K);
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

}

// Products whose k extent is a whole number of k-tiles (and whose operands
// meet the alignment gemm_prepare checks): operand tiles go from global
// memory straight into LDS by buffer loads with the LDS destination (no
// register staging, no LDS store instructions), double-buffered.  Each wave
// fills 8 rows per load (64 lanes x 16 bytes = 1 KB of LDS, written
// contiguously); rows past M or N read as zero through the buffer's range
// check.  LDS rows are 128 bytes without padding; chunk c of row r sits in
// slot c ^ ((r / 2) mod 8).  A 16-byte LDS read serves 16 lanes (256 bytes,
// all 64 banks) per pass; the 16 lanes read 16 consecutive rows, whose
// (row mod 2, slot) pairs are then all distinct: no bank conflict (keying
// on r mod 8 made rows r and r + 8 collide, halving LDS throughput).
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

template <int ET, int BM, int BN, bool SYM>
__device__ __forceinline__ void gemm_tile_direct(const GemmArgs &g, int bi, int bj, uint8_t *smem,
                                                 floatx16 (&acc)[BM / 64][BN / 64], const int tid = (int)threadIdx.x) {
    typedef typename Op<ET>::T T;
    constexpr int EPC = Op<ET>::EPC;
    constexpr int ESZ = (int)sizeof(T);
    constexpr int BK = 8 * EPC;
    constexpr int TM = BM / 64, TN = BN / 64;
    constexpr int RA = BM / 32, RB = BN / 32;
    constexpr bool SPLIT = ET == OP_BF16X3;
    // Split bf16 on tiles up to 128: both planes of a k-tile share one stage
    // and each fragment pair feeds the three products hi.hi, hi.lo, lo.hi (one
    // pass over k).  Larger tiles (two planes would not fit twice in LDS) run
    // three virtual k segments with planes (hi, hi, lo) for A, (hi, lo, hi)
    // for B.
    constexpr bool FUSED = TileShape<ET, BM, BN>::FUSED_SPLIT;
    constexpr int PLANE = (BM + BN) * 128;
    constexpr int STAGE = FUSED ? 2 * PLANE : PLANE;
    const int i0 = bi * BM, j0 = bj * BN;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const uint32_t abytes = (uint32_t)((int64_t)g.M * g.lda * ESZ), bbytes = (uint32_t)((int64_t)g.N * g.ldb * ESZ);
    const __amdgpu_buffer_rsrc_t ra_hi = make_rsrc(g.A, abytes), rb_hi = make_rsrc(g.B, bbytes);
    const __amdgpu_buffer_rsrc_t ra_lo = SPLIT ? make_rsrc((const T *)g.A + g.a_plane, abytes) : ra_hi;
    const __amdgpu_buffer_rsrc_t rb_lo = SPLIT ? make_rsrc((const T *)g.B + g.b_plane, bbytes) : rb_hi;
    const int lrow = lane >> 3, lslot = lane & 7;
    // global chunk this lane fetches into slot lslot of tile row
    // 8 (wave + 4p) + lrow: slot = chunk ^ ((row / 2) mod 8), and
    // (row / 2) mod 8 = (4 (wave mod 2) + lrow / 2) mod 8 for every p
    const int lchunk = lslot ^ ((4 * (wave & 1) + (lrow >> 1)) & 7);
    const int nfull = g.K / BK;                // whole k-tiles
    const int nkt = (g.K + BK - 1) / BK;       // k-tiles per segment
    const int nk = (SPLIT && !FUSED) ? 3 * nkt : nkt;

    // R x 8 rows of a tile, one 16-byte chunk per lane and row, straight to LDS
    auto direct_rows = [&](const __amdgpu_buffer_rsrc_t &rs, int64_t ld, int row0, uint32_t kb, uint8_t *dst,
                           auto nrep) {
#pragma unroll
        for (int p = 0; p < decltype(nrep)::value; ++p) {
            const int r0 = 8 * (wave + 4 * p);  // first of the 8 rows this wave fills
            const uint32_t off = (uint32_t)((row0 + r0 + lrow) * ld * ESZ) + kb;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(dst + r0 * 128), 16, off, 0, 0, 0);
        }
    };
    // ragged last k-tile: element-masked register loads (zero beyond K),
    // written to the same swizzled slots
    auto masked_rows = [&](const T *P, int64_t ld, int row0, int rows, int k, uint8_t *dst, auto nrep) {
#pragma unroll
        for (int p = 0; p < decltype(nrep)::value; ++p) {
            const int r = 8 * (wave + 4 * p) + lrow;
            *(u32x4 *)(dst + r * 128 + lslot * 16) = load_chunk_masked<ET>(P, ld, row0 + r, rows, k, g.K);
        }
    };
    const std::integral_constant<int, RA> na{};
    const std::integral_constant<int, RB> nb{};
    auto issue = [&](int kv, int stage) {
        int seg = 0, kt = kv;
        if constexpr (SPLIT && !FUSED) {
            seg = kv / nkt;
            kt = kv - seg * nkt;
        }
        uint8_t *base = smem + stage * STAGE;
        if (kt < nfull) {
            const uint32_t kb = (uint32_t)kt * BK * ESZ + lchunk * 16;
            direct_rows(SPLIT && seg == 2 ? ra_lo : ra_hi, g.lda, i0, kb, base, na);
            direct_rows(SPLIT && seg == 1 ? rb_lo : rb_hi, g.ldb, j0, kb, base + BM * 128, nb);
            if constexpr (FUSED) {
                direct_rows(ra_lo, g.lda, i0, kb, base + PLANE, na);
                direct_rows(rb_lo, g.ldb, j0, kb, base + PLANE + BM * 128, nb);
            }
        } else {
            const T *A = (const T *)g.A, *B = (const T *)g.B;
            const int k = kt * BK + lchunk * EPC;
            masked_rows(A + (SPLIT && seg == 2 ? g.a_plane : 0), g.lda, i0, g.M, k, base, na);
            masked_rows(B + (SPLIT && seg == 1 ? g.b_plane : 0), g.ldb, j0, g.N, k, base + BM * 128, nb);
            if constexpr (FUSED) {
                masked_rows(A + g.a_plane, g.lda, i0, g.M, k, base + PLANE, na);
                masked_rows(B + g.b_plane, g.ldb, j0, g.N, k, base + PLANE + BM * 128, nb);
            }
        }
    };
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    // fragment rows are 16-row aligned plus frow: the row's swizzle key
    // is (frow / 2) mod 8
    const int frow = lane & 31, fh = lane >> 5, sw = (frow >> 1) & 7;
    auto compute = [&](int stage) {
        const uint8_t *As = smem + stage * STAGE + (wm * (BM / 2)) * 128;
        const uint8_t *Bs = smem + stage * STAGE + BM * 128 + (wn * (BN / 2)) * 128;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c0 = ((fh * 4 + q * 2) ^ sw) * 16, c1 = ((fh * 4 + q * 2 + 1) ^ sw) * 16;
            u32x4 af[TM][2], bf[TN][2];
#pragma unroll
            for (int a = 0; a < TM; ++a) {
                af[a][0] = *(const u32x4 *)&As[(a * 32 + frow) * 128 + c0];
                af[a][1] = *(const u32x4 *)&As[(a * 32 + frow) * 128 + c1];
            }
#pragma unroll
            for (int b = 0; b < TN; ++b) {
                bf[b][0] = *(const u32x4 *)&Bs[(b * 32 + frow) * 128 + c0];
                bf[b][1] = *(const u32x4 *)&Bs[(b * 32 + frow) * 128 + c1];
            }
            if constexpr (FUSED) {
                u32x4 al[TM][2], bl[TN][2];
#pragma unroll
                for (int a = 0; a < TM; ++a) {
                    al[a][0] = *(const u32x4 *)&As[PLANE + (a * 32 + frow) * 128 + c0];
                    al[a][1] = *(const u32x4 *)&As[PLANE + (a * 32 + frow) * 128 + c1];
                }
#pragma unroll
                for (int b = 0; b < TN; ++b) {
                    bl[b][0] = *(const u32x4 *)&Bs[PLANE + (b * 32 + frow) * 128 + c0];
                    bl[b][1] = *(const u32x4 *)&Bs[PLANE + (b * 32 + frow) * 128 + c1];
                }
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b) {
                        acc[a][b] = mfma_32b<ET>(af[a][0], af[a][1], bf[b][0], bf[b][1], acc[a][b]);
                        acc[a][b] = mfma_32b<ET>(af[a][0], af[a][1], bl[b][0], bl[b][1], acc[a][b]);
                        acc[a][b] = mfma_32b<ET>(al[a][0], al[a][1], bf[b][0], bf[b][1], acc[a][b]);
                    }
            } else {
#pragma unroll
                for (int a = 0; a < TM; ++a)
#pragma unroll
                    for (int b = 0; b < TN; ++b)
                        acc[a][b] = mfma_32b<ET>(af[a][0], af[a][1], bf[b][0], bf[b][1], acc[a][b]);
            }
        }
    };
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) issue(kt + 1, (kt + 1) & 1);
        compute(kt & 1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

// Block-uniform values read from memory: every lane reads the same words,
// and readfirstlane keeps them in scalar registers (the descriptor of a
// device-described product then costs no vector registers).
template <typename T>
__device__ __forceinline__ T uniform_load(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T out;
    const uint32_t *src = (const uint32_t *)p;
    uint32_t *dst = (uint32_t *)&out;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return out;
}

// owner_of (batched.h) with block-uniform control flow.
__device__ __forceinline__ int owner_of_uniform(const int *prefix, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(prefix[mid]) <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One block tile of a product: the operand body (direct-to-LDS or
// register-staged, chosen per product) accumulates, then one epilogue.
template <int ET, int BM, int BN, bool TWO_A, bool SYM>
__device__ __forceinline__ void gemm_block(const GemmArgs &g, int bi, int bj, uint8_t *smem,
                                           const int tid = (int)threadIdx.x) {
    floatx16 acc[BM / 64][BN / 64];
    bool done = false;
    if constexpr (!TWO_A) {
        if (g.direct) {
            gemm_tile_direct<ET, BM, BN, SYM>(g, bi, bj, smem, acc, tid);
            done = true;
        }
    }
    if (!done) gemm_tile<ET, BM, BN, TWO_A, SYM>(g, bi, bj, smem, acc, tid);
    store_tile<BM, BN, SYM>(g, bi, bj, acc, smem, tid);
}

// One product: block b computes local tile xcd_remap(b) (each XCD gets a
// contiguous range of tiles, so tiles sharing panels share an L2).
template <int ET, int BM, int BN, int OCC, bool TWO_A, bool SYM>
__global__ __launch_bounds__(256, OCC) void gemm_nt(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileShape<ET, BM, BN>::SMEM];
    int bi, bj;
    tile_coords<SYM>(xcd_remap(blockIdx.x, gridDim.x), g.M, g.N, BM, BN, bi, bj);
    gemm_block<ET, BM, BN, TWO_A, SYM>(g, bi, bj, smem);
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
    // a copy: the fields then live in registers for the whole tile instead
    // of being re-read from the descriptor table after every store
    const GemmArgs g = args[lo];
    int bi, bj;
    tile_coords<SYM>(b - prefix[lo], g.M, g.N, BM, BN, bi, bj);
    gemm_block<ET, BM, BN, TWO_A, SYM>(g, bi, bj, smem);
}

// One stage of a device-described batch (psvt_svt_batched): a fixed grid of
// blocks loops over the stage's tiles of every matrix whose model picks this
// configuration (the prefix sum of its count class); each tile's descriptor
// is rebuilt from the stage template and the matrix's record, in registers.
// The tiles are computed exactly as in a single call.
template <int ET, int BM, int BN, int OCC, bool TWO_A, bool SYM>
__global__ __launch_bounds__(256, OCC) void gemm_batched(BatchView v, GemmStageT st) {
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileShape<ET, BM, BN>::SMEM];
    const int total = __builtin_amdgcn_readfirstlane(v.prefix[v.count]);
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
        const int i = owner_of_uniform(v.prefix, v.count, t);
        const MatInfo mi = uniform_load(&v.mats[i]);
        GemmArgs g;
        relocate_gemm(st, mi, v.op, v.lp, g);
        int bi, bj;
        tile_coords<SYM>(t - __builtin_amdgcn_readfirstlane(v.prefix[i]), g.M, g.N, BM, BN, bi, bj);
        // the thread index as an opaque value of this iteration: the bodies'
        // per-thread offsets are then recomputed per tile instead of being
        // hoisted out of the loop and held in registers across it
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        gemm_block<ET, BM, BN, TWO_A, SYM>(g, bi, bj, smem, tid);
        __syncthreads();  // the next tile refills LDS
    }
}

// ------------------------------------------------------------ launchers
// Launchers of one tile configuration (instantiated one operand type and
// configuration per translation unit) and the dispatchers over them.

template <int ET, int BM, int OCC>
hipError_t gemm_launch_bm(const GemmArgs &g, int nblocks, hipStream_t st) {
    if (g.sym)
        hipLaunchKernelGGL((gemm_nt<ET, BM, BM, OCC, false, true>), dim3(nblocks), dim3(256), 0, st, g);
    else if (ET == OP_F32 && g.A2)
        hipLaunchKernelGGL((gemm_nt<ET, BM, BM, OCC, ET == OP_F32, false>), dim3(nblocks), dim3(256), 0, st, g);
    else
        hipLaunchKernelGGL((gemm_nt<ET, BM, BM, OCC, false, false>), dim3(nblocks), dim3(256), 0, st, g);
    return hipGetLastError();
}

// blocks per CU a configuration targets (LDS-limited: 160 KB per CU)
template <int ET, int BM>
constexpr int tile_occupancy() {
    return (160 * 1024) / TileShape<ET, BM, BM>::SMEM < 4 ? (160 * 1024) / TileShape<ET, BM, BM>::SMEM : 4;
}

template <int ET>
hipError_t gemm_launch(const GemmArgs &g, int tile, int nblocks, hipStream_t st) {
    switch (tile) {
        case 1: return gemm_launch_bm<ET, 64, tile_occupancy<ET, 64>()>(g, nblocks, st);
        case 3: return gemm_launch_bm<ET, 192, 1>(g, nblocks, st);
        case 4: return gemm_launch_bm<ET, 256, 1>(g, nblocks, st);
        default: return gemm_launch_bm<ET, 128, tile_occupancy<ET, 128>()>(g, nblocks, st);
    }
}

template <int ET, int BM, int OCC>
hipError_t gemm_grouped_bm(const GemmArgs *args, const int *prefix, int n, int total, int sym, int two_a,
                           hipStream_t st) {
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

template <int ET, int BM, int OCC>
hipError_t gemm_batched_bm(const BatchView &v, const GemmStageT &s, int grid, hipStream_t st) {
    if (s.g.sym)
        hipLaunchKernelGGL((gemm_batched<ET, BM, BM, OCC, false, true>), dim3(grid), dim3(256), 0, st, v, s);
    else if (ET == OP_F32 && s.r.p[1] != PC_NULL)
        hipLaunchKernelGGL((gemm_batched<ET, BM, BM, OCC, ET == OP_F32, false>), dim3(grid), dim3(256), 0, st, v, s);
    else
        hipLaunchKernelGGL((gemm_batched<ET, BM, BM, OCC, false, false>), dim3(grid), dim3(256), 0, st, v, s);
    return hipGetLastError();
}

// blocks a batched stage launches for configuration `tile`: the
// configuration's blocks per CU on every CU
template <int ET>
int gemm_batched_grid(int tile) {
    switch (tile) {
        case 1: return 256 * tile_occupancy<ET, 64>();
        case 3: return 256;
        case 4: return 256;
        default: return 256 * tile_occupancy<ET, 128>();
    }
}

template <int ET>
hipError_t gemm_launch_batched(const BatchView &v, const GemmStageT &s, int tile, hipStream_t st) {
    const int grid = gemm_batched_grid<ET>(tile);
    switch (tile) {
        case 1: return gemm_batched_bm<ET, 64, tile_occupancy<ET, 64>()>(v, s, grid, st);
        case 3: return gemm_batched_bm<ET, 192, 1>(v, s, grid, st);
        case 4: return gemm_batched_bm<ET, 256, 1>(v, s, grid, st);
        default: return gemm_batched_bm<ET, 128, tile_occupancy<ET, 128>()>(v, s, grid, st);
    }
}

template <int ET>
hipError_t gemm_launch_grouped(const GemmArgs *args, const int *prefix, int n, int total, int tile, int sym,
                               int two_a, hipStream_t st) {
    switch (tile) {
        case 1: return gemm_grouped_bm<ET, 64, tile_occupancy<ET, 64>()>(args, prefix, n, total, sym, two_a, st);
        case 3: return gemm_grouped_bm<ET, 192, 1>(args, prefix, n, total, sym, two_a, st);
        case 4: return gemm_grouped_bm<ET, 256, 1>(args, prefix, n, total, sym, two_a, st);
        default: return gemm_grouped_bm<ET, 128, tile_occupancy<ET, 128>()>(args, prefix, n, total, sym, two_a, st);
    }
}

}  // namespace psvt
