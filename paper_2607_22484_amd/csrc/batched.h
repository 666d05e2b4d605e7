// Device-described batches (psvt_svt_batched): the per-matrix record the
// setup kernel writes, and the relocation of a template stage to one
// matrix.
//
// The host plans the method once for a template matrix (sentinel pointers,
// distinct sizes) and records, for every field of every stage that depends
// on the matrix, where it comes from: a pointer is the input A, the output
// Y, the matrix's status word, or one of its workspace buffers (layout.h);
// its row stride and split-bf16 plane stride follow from that buffer; a
// size is l, s (the long and short side), m or n; tau is the matrix's.  A
// block rebuilds the stage's descriptor for its matrix in registers from
// the template and the matrix's record.  The same functions run on the host,
// which checks them against plans of probe matrices before any launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "layout.h"
#include "tilemodel.h"

namespace psvt {

// One matrix of a device-described batch (written by the setup kernel).
struct MatInfo {
    const float *A;
    float *Y;
    uint32_t *status;
    int64_t m, n, lda, ldy, l, s;
    double tau;
    char *base;  // this matrix's workspace
    int right;   // right-sided (A^T A) or left-sided (A A^T)
    int valid;   // 0: descriptor rejected or workspace exhausted (skipped)
};

// Where a pointer field comes from.
enum PtrCode : uint8_t { PC_NULL = 0, PC_A = 1, PC_Y = 2, PC_STATUS = 3, PC_BUF = 16 /* + BufId */ };
// Where a size field comes from.
enum DimCode : uint8_t { DC_LIT = 0, DC_L = 1, DC_S = 2, DC_M = 3, DC_N = 4 };
// Plane strides: copied (0) or the plane of the pointer's buffer (1).
enum PlaneCode : uint8_t { PL_LIT = 0, PL_BUF = 1 };

// Gemm pointers in this order: A, A2, B, D, C, CT, Clp, CTlp.
struct GemmReloc {
    uint8_t p[8];
    uint8_t pl[4];  // a_plane (A), b_plane (B), lp_plane (Clp), lp_plane_t (CTlp)
    uint8_t M, N, K;
    uint8_t wa2_tau;  // wa2 = -tau
    uint8_t sc;       // sc = the matrix's scalar block
    uint8_t swap_y;   // the output Y: row-major in C for right-sided, transposed in CT for left-sided
    uint8_t right_t;  // the template's side: C and CT swap for a matrix of the other side
};
struct NormReloc {
    uint8_t X, part, sc, status, rows, cols, tau;
};
struct TileReloc {
    uint8_t X, Y, YT, L, sc, rows, cols, lplane, swap_t;  // swap_t: Y <-> YT for a matrix of the other side
    uint8_t right_t;                                      // the template's side
};

struct GemmStageT {
    GemmArgs g;
    GemmReloc r;
    int dtype;
};
struct NormStageT {
    NormOp n;
    NormReloc r;
};
struct TileStageT {
    TileOp t;
    TileReloc r;
};

// What a stage launch sees of the batch: the records and the prefix sum of
// its count class (count + 1 entries; entry count = the launch's total).
struct BatchView {
    const MatInfo *mats;
    const int *prefix;
    int count;
    int op, lp;  // layout parameters shared by the batch
};

__host__ __device__ inline Layout mat_layout(const MatInfo &mi, int op, int lp) {
    return layout_for(op, mi.l, mi.s, mi.right != 0, lp != 0, false);
}

__host__ __device__ inline void *reloc_ptr(uint8_t code, const MatInfo &mi, const Layout &L) {
    switch (code) {
        case PC_NULL: return nullptr;
        case PC_A: return (void *)mi.A;
        case PC_Y: return mi.Y;
        case PC_STATUS: return mi.status;
        default: return mi.base + L.offset(code - PC_BUF);
    }
}
__host__ __device__ inline int64_t reloc_ld(uint8_t code, int64_t lit, const MatInfo &mi, const Layout &L) {
    switch (code) {
        case PC_NULL: case PC_STATUS: return lit;
        case PC_A: return mi.lda;
        case PC_Y: return mi.ldy;
        default: return L.ld(code - PC_BUF);
    }
}
__host__ __device__ inline int64_t reloc_plane(uint8_t plcode, uint8_t ptrcode, int64_t lit, const Layout &L) {
    return (plcode == PL_BUF && ptrcode >= PC_BUF) ? L.plane(ptrcode - PC_BUF) : lit;
}
__host__ __device__ inline int64_t reloc_dim(uint8_t code, int64_t lit, const MatInfo &mi) {
    switch (code) {
        case DC_L: return mi.l;
        case DC_S: return mi.s;
        case DC_M: return mi.m;
        case DC_N: return mi.n;
        default: return lit;
    }
}

__host__ __device__ inline void relocate_gemm(const GemmStageT &st, const MatInfo &mi, int op, int lp,
                                              GemmArgs &g) {
    const Layout L = mat_layout(mi, op, lp);
    const GemmReloc &r = st.r;
    g = st.g;
    g.A = reloc_ptr(r.p[0], mi, L);
    g.lda = reloc_ld(r.p[0], g.lda, mi, L);
    g.A2 = reloc_ptr(r.p[1], mi, L);
    g.lda2 = reloc_ld(r.p[1], g.lda2, mi, L);
    g.B = reloc_ptr(r.p[2], mi, L);
    g.ldb = reloc_ld(r.p[2], g.ldb, mi, L);
    g.D = (const float *)reloc_ptr(r.p[3], mi, L);
    g.ldd = reloc_ld(r.p[3], g.ldd, mi, L);
    g.C = (float *)reloc_ptr(r.p[4], mi, L);
    g.ldc = reloc_ld(r.p[4], g.ldc, mi, L);
    g.CT = (float *)reloc_ptr(r.p[5], mi, L);
    g.ldct = reloc_ld(r.p[5], g.ldct, mi, L);
    g.Clp = reloc_ptr(r.p[6], mi, L);
    g.ldclp = reloc_ld(r.p[6], g.ldclp, mi, L);
    g.CTlp = reloc_ptr(r.p[7], mi, L);
    g.ldctlp = reloc_ld(r.p[7], g.ldctlp, mi, L);
    g.a_plane = reloc_plane(r.pl[0], r.p[0], g.a_plane, L);
    g.b_plane = reloc_plane(r.pl[1], r.p[2], g.b_plane, L);
    g.lp_plane = reloc_plane(r.pl[2], r.p[6], g.lp_plane, L);
    g.lp_plane_t = reloc_plane(r.pl[3], r.p[7], g.lp_plane_t, L);
    g.M = (int)reloc_dim(r.M, g.M, mi);
    g.N = (int)reloc_dim(r.N, g.N, mi);
    g.K = (int)reloc_dim(r.K, g.K, mi);
    if (r.wa2_tau) g.wa2 = (float)(-mi.tau);
    if (r.sc) g.sc = (const Scalars *)(mi.base + L.scal);
    if (r.swap_y && (mi.right != 0) != (r.right_t != 0)) {  // Y transposed: the other side's view
        float *c = g.C;
        const int64_t ldc = g.ldc;
        g.C = g.CT;
        g.ldc = g.ldct;
        g.CT = c;
        g.ldct = ldc;
    }
    gemm_prepare(g, st.dtype);
}

__host__ __device__ inline void relocate_norm(const NormStageT &st, const MatInfo &mi, int op, int lp, NormOp &n) {
    const Layout L = mat_layout(mi, op, lp);
    const NormReloc &r = st.r;
    n = st.n;
    n.X = (const float *)reloc_ptr(r.X, mi, L);
    n.ld = reloc_ld(r.X, n.ld, mi, L);
    n.rows = reloc_dim(r.rows, n.rows, mi);
    n.cols = reloc_dim(r.cols, n.cols, mi);
    if (r.part) n.part = (double *)(mi.base + L.part);
    if (r.sc) n.sc = (Scalars *)(mi.base + L.scal);
    if (r.status) n.status = mi.status;
    if (r.tau) n.tau = mi.tau;
    n.nparts = norm_parts(n.rows, n.cols);
}

__host__ __device__ inline void relocate_tile(const TileStageT &st, const MatInfo &mi, int op, int lp, TileOp &t) {
    const Layout L = mat_layout(mi, op, lp);
    const TileReloc &r = st.r;
    t = st.t;
    t.X = (const float *)reloc_ptr(r.X, mi, L);
    t.ldx = reloc_ld(r.X, t.ldx, mi, L);
    t.Y = (float *)reloc_ptr(r.Y, mi, L);
    t.ldy = reloc_ld(r.Y, t.ldy, mi, L);
    t.YT = (float *)reloc_ptr(r.YT, mi, L);
    t.ldyt = reloc_ld(r.YT, t.ldyt, mi, L);
    t.L = reloc_ptr(r.L, mi, L);
    t.ldl = reloc_ld(r.L, t.ldl, mi, L);
    t.lplane = reloc_plane(r.lplane, r.L, t.lplane, L);
    t.rows = reloc_dim(r.rows, t.rows, mi);
    t.cols = reloc_dim(r.cols, t.cols, mi);
    if (r.sc) t.sc = (const Scalars *)(mi.base + L.scal);
    if (r.swap_t && (mi.right != 0) != (r.right_t != 0)) {
        float *y = t.Y;
        const int64_t ldy = t.ldy;
        t.Y = t.YT;
        t.ldy = t.ldyt;
        t.YT = y;
        t.ldyt = ldy;
    }
}

// Last index i in [0, n) with prefix[i] <= t (the matrix that owns item t:
// matrices with no items share their prefix value with the next one).
__host__ __device__ inline int owner_of(const int *prefix, int n, int t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Count classes: what a stage launch enumerates per matrix.
enum CountKind { CK_GEMM = 0, CK_NORM = 1, CK_TILE = 2 };
struct CountClass {
    int kind;
    int dtype, sym, tile;     // CK_GEMM: tiles of configuration `tile` when the model picks it
    uint8_t c0, c1, c2;       // dim codes: M, N, K (gemm); rows, cols (norm, tile)
    int lit0, lit1, lit2;     // their literal values when coded DC_LIT
    int group;                // CK_TILE: 64 x 64 tiles per item (>= 1)
};

__host__ __device__ inline int class_count(const CountClass &c, const MatInfo &mi, const TileModelTable &model) {
    if (!mi.valid) return 0;
    const int64_t d0 = reloc_dim(c.c0, c.lit0, mi), d1 = reloc_dim(c.c1, c.lit1, mi), d2 = reloc_dim(c.c2, c.lit2, mi);
    if (c.kind == CK_GEMM) {
        if (d0 <= 0 || d1 <= 0) return 0;
        if (pick_tile(model, c.dtype, (int)d0, (int)d1, (int)d2, c.sym) != c.tile) return 0;
        return tile_count((int)d0, (int)d1, c.sym, tile_bm(c.tile));
    }
    if (c.kind == CK_NORM) return norm_parts(d0, d1);
    const int64_t tiles = ((d0 + 63) / 64) * ((d1 + 63) / 64);
    return (int)((tiles + c.group - 1) / c.group);
}

// ----------------------------------------------- persistent executor
// PSVT_FLAG_PERSISTENT runs a batch's stages in ONE launch: blocks take
// tickets in (launch, item) order, where a launch is what the per-stage
// form would launch (a stage, or one tile configuration of a product stage)
// and its items are the prefix sum of its count class.  Matrix i's item of
// launch j waits until matrix i has completed every item of launches < j;
// those hold lower tickets, taken by running blocks, so the lowest
// unfinished ticket can always run and the launch drains.  Waits are
// bounded: past the bound a block raises the abort flag, every later item
// is skipped, and the kernel still ends.

// 64 x 64 elementwise tiles per item of the persistent executor.
constexpr int kPersistTileGroup = 8;

// A template stage as the persistent kernel reads it.
struct StageT {
    int kind, dtype;
    union {
        GemmStageT g;
        NormStageT n;
        TileStageT t;
    };
};

// One launch of the per-stage form: its stage, count class (-1: the final
// pass of a norm, one item per matrix) and tile configuration.
struct PLaunch {
    int32_t stage;
    int16_t cls;
    int8_t tile, final_pass;  // tile: gemm configuration, or tile-op tiles per item
};

// At byte 0 of the workspace of a persistent call: the ticket counter and the
// abort flag (nonzero after the call: a wait passed its bound, results and
// status words of unfinished matrices are invalid).
struct PersistCtl {
    uint32_t ticket, abort;
    uint32_t pad[62];
};

struct PersistArgs {
    const MatInfo *mats;
    int count, op, lp, status_on;
    const int *prefix;  // count classes' prefix sums, count + 1 entries each
    const PLaunch *launches;
    int nl;
    const StageT *stages;
    int *lbase;  // nl + 1: first ticket of each launch
    int *deps;   // count x nl: items of matrix i in launches < j
    int *done;   // count: items of matrix i completed
    PersistCtl *ctl;
    long long spin_limit;
};

// Items of matrix i in launch L (count classes' prefix sums, count + 1 each).
__host__ __device__ inline int persist_items(const PLaunch &L, const int *prefix, int count, int i) {
    if (L.final_pass) return 1;
    const int *pre = prefix + (size_t)L.cls * ((size_t)count + 1);
    return pre[i + 1] - pre[i];
}
// All items of launch L.
__host__ __device__ inline int persist_launch_items(const PLaunch &L, const int *prefix, int count) {
    return L.final_pass ? count : prefix[(size_t)L.cls * ((size_t)count + 1) + count];
}
// Ticket T -> launch j, matrix i, item within the matrix's share of the launch.
__host__ __device__ inline void persist_decode(const int *lbase, int nl, const PLaunch *launches, const int *prefix,
                                               int count, int T, int &j, int &i, int &item) {
    j = owner_of(lbase, nl, T);
    const PLaunch L = launches[j];
    const int t = T - lbase[j];
    i = t;
    item = 0;
    if (!L.final_pass) {
        const int *pre = prefix + (size_t)L.cls * ((size_t)count + 1);
        i = owner_of(pre, count, t);
        item = t - pre[i];
    }
}

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st);
hipError_t launch_persistent(const PersistArgs &a, hipStream_t st);

}  // namespace psvt
