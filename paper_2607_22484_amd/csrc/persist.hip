// The persistent executor of device-described batches (PSVT_FLAG_PERSISTENT):
// one launch runs every stage of every matrix (batched.h explains the ticket
// order and why it drains).  Each item is computed by the same device body,
// on the same relocated descriptor, as in the per-stage form, so results are
// bitwise those of single calls that use the same tile configurations.
//
// Memory ordering between blocks: a block that completes an item makes its
// stores visible at agent scope (each wave waits for its stores, then one
// release fence, then the counter increment); a block that has waited for a
// counter takes an acquire fence before the barrier after which its waves
// read what the item depends on.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/psvt.h"
#include "batched.h"
#include "bodies.h"
#include "kernels.h"
#include "plan.h"
#include "tile.h"

namespace psvt {
namespace {

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// LDS: the largest tile body of the executor's tile set, the norm
// reduction, the elementwise 64 x 64 tile.
constexpr int kPersistSmem =
    cmax(cmax(cmax(TileShape<OP_F32, 128, 128>::SMEM, TileShape<OP_BF16, 128, 128>::SMEM),
              cmax(TileShape<OP_FP8, 64, 64>::SMEM, TileShape<OP_BF16X3, 64, 64>::SMEM)),
         cmax(64 * 65 * (int)sizeof(float), 256 * (int)sizeof(double)));
static_assert(kPersistMaxTile[OP_F32] == 2 && kPersistMaxTile[OP_BF16] == 2 && kPersistMaxTile[OP_FP8] == 1 &&
                  kPersistMaxTile[OP_BF16X3] == 1,
              "the executor instantiates exactly this tile set");
static_assert(2 * (kPersistSmem + 64) <= 160 * 1024, "two blocks per CU");
constexpr int kPersistBlocksPerCU = 2;

constexpr int kUploadWords = 960;
struct UploadArgs {
    uint32_t *dst;
    uint32_t words;
    uint32_t data[kUploadWords];
};

__global__ __launch_bounds__(256) void upload_words(UploadArgs a) {
    for (uint32_t i = threadIdx.x; i < a.words; i += blockDim.x) a.dst[i] = a.data[i];
}

// First ticket of every launch, the per-matrix dependency counts, and
// cleared counters (a kernel, not a memset: the call may be captured).
__global__ __launch_bounds__(1024) void persist_setup(PersistArgs a) {
    if (threadIdx.x == 0) {
        int run = 0;
        for (int j = 0; j < a.nl; ++j) {
            a.lbase[j] = run;
            run += persist_launch_items(a.launches[j], a.prefix, a.count);
        }
        a.lbase[a.nl] = run;
        a.ctl->ticket = 0u;
        a.ctl->abort = 0u;
    }
    for (int i = threadIdx.x; i < a.count; i += blockDim.x) {
        a.done[i] = 0;
        int run = 0;
        for (int j = 0; j < a.nl; ++j) {
            a.deps[(size_t)i * a.nl + j] = run;
            run += persist_items(a.launches[j], a.prefix, a.count, i);
        }
    }
}

__device__ __forceinline__ uint32_t load_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_agent(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Raise the abort flag; with status words, mark every matrix invalid (a
// matrix whose status stage still completes writes its own, valid, word).
// Wave 0, all lanes (they store the same values).
__device__ void abort_batch(const PersistArgs &a) {
    __hip_atomic_store(&a.ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!a.status_on) return;
    for (int i = 0; i < a.count; ++i)
        if (a.mats[i].status) *a.mats[i].status = PSVT_STATUS_INVALID;
}

// Wave 0 of a block, all lanes (every branch and loop condition is
// wave-uniform): 0 = skip (aborted), 1 = run (no dependency), 2 = run after
// an acquire (the matrix's earlier items are complete).
__device__ int wait_ready(const PersistArgs &a, int i, int want) {
    if (__builtin_amdgcn_readfirstlane(load_agent(&a.ctl->abort))) return 0;
    if (want == 0) return 1;
    long long n = 0;
    while (__builtin_amdgcn_readfirstlane(load_agent(&a.done[i])) < want) {
        if (n++ >= a.spin_limit) {
            abort_batch(a);
            return 0;
        }
        if (__builtin_amdgcn_readfirstlane(load_agent(&a.ctl->abort))) return 0;
        __builtin_amdgcn_s_sleep(16);
    }
    // acquire at agent scope: this CU's L1 and the L2 drop stale lines, for
    // every wave of the block (they read only after the barrier that follows)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return 2;
}

// Add `one` (1 in lane 0, 0 elsewhere) from every lane of a wave: the word
// grows by 1, and lane 0 reads the value before its add (adds of 0 change
// nothing), whatever the order of the lanes' atomics.
__device__ __forceinline__ uint32_t wave_inc(uint32_t *p, uint32_t one) {
    return __builtin_amdgcn_readfirstlane(atomicAdd(p, one));
}

// The block's LDS: the launch's dynamic shared memory (kPersistSmem bytes),
// named in each item function so that the tile bodies, inlined there, keep
// LDS addressing.
extern __shared__ __attribute__((aligned(16))) uint8_t persist_lds[];

template <int ET, int BM>
__device__ __forceinline__ void gemm_item(const GemmArgs &g, bool two_a, int item, uint8_t *smem) {
    int bi, bj;
    floatx16 acc[BM / 64][BM / 64];
    if (g.sym) {
        tile_coords<true>(item, g.M, g.N, BM, BM, bi, bj);
        if (g.direct)
            gemm_tile_direct<ET, BM, BM, true>(g, bi, bj, smem, acc);
        else
            gemm_tile<ET, BM, BM, false, true>(g, bi, bj, smem, acc);
        store_tile<BM, BM, true>(g, bi, bj, acc, smem);
        return;
    }
    tile_coords<false>(item, g.M, g.N, BM, BM, bi, bj);
    bool done = false;
    if constexpr (ET == OP_F32) {
        if (two_a) {
            gemm_tile<ET, BM, BM, true, false>(g, bi, bj, smem, acc);
            done = true;
        }
    }
    if (!done) {
        if (g.direct)
            gemm_tile_direct<ET, BM, BM, false>(g, bi, bj, smem, acc);
        else
            gemm_tile<ET, BM, BM, false, false>(g, bi, bj, smem, acc);
    }
    store_tile<BM, BM, false>(g, bi, bj, acc, smem);
}

// One item per call, not inlined: each configuration gets its own register
// allocation (one kernel holding all of them inline spills heavily).
template <int ET, int BM>
__device__ __attribute__((noinline)) void gemm_call(const StageT *S, const MatInfo *mip, int op, int lp, int item) {
    const MatInfo mi = *mip;
    GemmArgs g;
    relocate_gemm(S->g, mi, op, lp, g);
    gemm_item<ET, BM>(g, S->g.r.p[1] != PC_NULL, item, persist_lds);
}

__device__ __attribute__((noinline)) void norm_call(const StageT *S, const MatInfo *mip, int op, int lp, int item,
                                                    int final_pass) {
    const MatInfo mi = *mip;
    NormOp n;
    relocate_norm(S->n, mi, op, lp, n);
    if (final_pass) {
        if (mi.valid) fro_final_body(n, (double *)persist_lds);
    } else {
        fro_partial_body(n, item, (double *)persist_lds);
    }
}

// Tiles [item * group, (item + 1) * group) of an elementwise stage.
__device__ __attribute__((noinline)) void tile_call(const StageT *S, const MatInfo *mip, int op, int lp, int item,
                                                    int group) {
    const MatInfo mi = *mip;
    TileOp t;
    relocate_tile(S->t, mi, op, lp, t);
    const int tiles = __builtin_amdgcn_readfirstlane((int)(((t.rows + 63) / 64) * ((t.cols + 63) / 64)));
    const int t0 = item * group, t1 = t0 + group < tiles ? t0 + group : tiles;
    for (int k = t0; k < t1; ++k) {
        tile_op_body(t, k, (float(*)[65])persist_lds);
        __syncthreads();  // the next tile refills LDS
    }
}

// Returns false for a configuration outside the executor's tile set.
__device__ __forceinline__ bool run_item(const PersistArgs &a, const PLaunch &L, int i, int item) {
    const StageT *S = a.stages + L.stage;
    const MatInfo *mi = a.mats + i;
    const int kind = S->kind;
    if (kind == ST_GEMM) {
        switch (S->dtype * 8 + L.tile) {
            case OP_F32 * 8 + 1: gemm_call<OP_F32, 64>(S, mi, a.op, a.lp, item); return true;
            case OP_F32 * 8 + 2: gemm_call<OP_F32, 128>(S, mi, a.op, a.lp, item); return true;
            case OP_BF16 * 8 + 1: gemm_call<OP_BF16, 64>(S, mi, a.op, a.lp, item); return true;
            case OP_BF16 * 8 + 2: gemm_call<OP_BF16, 128>(S, mi, a.op, a.lp, item); return true;
            case OP_FP8 * 8 + 1: gemm_call<OP_FP8, 64>(S, mi, a.op, a.lp, item); return true;
            case OP_BF16X3 * 8 + 1: gemm_call<OP_BF16X3, 64>(S, mi, a.op, a.lp, item); return true;
            default: return false;
        }
    }
    if (kind == ST_NORM)
        norm_call(S, mi, a.op, a.lp, item, L.final_pass);
    else
        tile_call(S, mi, a.op, a.lp, item, L.tile);
    return true;
}

// Control flow around every barrier is wave-uniform: wave 0 (all its lanes)
// takes the ticket, waits, and counts the previous item done; values shared
// through LDS are read back with readfirstlane, so the loop exit is a scalar
// branch.  (A branch on threadIdx.x == 0 next to the loop's back edge lets
// the compiler move thread 0's work out of the loop the other lanes keep
// running: the waves then pass the barriers without it and re-read a ticket
// that never changes.)
__global__ __launch_bounds__(256, kPersistBlocksPerCU) void batched_persistent(PersistArgs a) {
    __shared__ int s_ticket, s_go;
    const int total = __builtin_amdgcn_readfirstlane(a.lbase[a.nl]);
    const bool wave0 = __builtin_amdgcn_readfirstlane((int)threadIdx.x) == 0;
    const uint32_t one = (threadIdx.x & 63) == 0 ? 1u : 0u;
    int prev = -1;  // matrix of this block's previous item
    for (;;) {
        if (wave0) {
            // the previous item is complete: count it (its stores were
            // released before the barrier that ended it), then take a ticket
            if (prev >= 0) wave_inc((uint32_t *)&a.done[prev], one);
            s_ticket = (int)wave_inc(&a.ctl->ticket, one);
        }
        __syncthreads();
        const int T = __builtin_amdgcn_readfirstlane(s_ticket);
        if (T >= total) break;
        int j, i, item;
        persist_decode(a.lbase, a.nl, a.launches, a.prefix, a.count, T, j, i, item);
        j = __builtin_amdgcn_readfirstlane(j);
        i = __builtin_amdgcn_readfirstlane(i);
        item = __builtin_amdgcn_readfirstlane(item);
        const PLaunch L = a.launches[j];
        if (wave0) s_go = wait_ready(a, i, __builtin_amdgcn_readfirstlane(a.deps[(size_t)i * a.nl + j]));
        __syncthreads();
        const int go = __builtin_amdgcn_readfirstlane(s_go);
        if (go) {
            const bool ok = run_item(a, L, i, item);
            if (!ok && wave0) abort_batch(a);
        }
        // release: every wave waits until its own stores have reached the
        // L2 (vmcnt 0), then, after the barrier, wave 0 alone writes the L2
        // back at agent scope (one write-back per item instead of one per
        // wave) before it counts the item done
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt unconstrained
        __syncthreads();                     // LDS is free for the next item, too
        if (wave0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        prev = i;
    }
}

}  // namespace

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes % 4) return hipErrorInvalidValue;
    const uint32_t *w = (const uint32_t *)src;
    size_t left = bytes / 4;
    uint32_t *d = (uint32_t *)dst;
    while (left) {
        UploadArgs a;
        a.dst = d;
        a.words = (uint32_t)(left < (size_t)kUploadWords ? left : (size_t)kUploadWords);
        for (uint32_t k = 0; k < a.words; ++k) a.data[k] = w[k];
        for (uint32_t k = a.words; k < (uint32_t)kUploadWords; ++k) a.data[k] = 0u;
        hipLaunchKernelGGL(upload_words, dim3(1), dim3(256), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        w += a.words;
        d += a.words;
        left -= a.words;
    }
    return hipSuccess;
}

hipError_t launch_persistent(const PersistArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(persist_setup, dim3(1), dim3(1024), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // more than 64 KB of dynamic LDS per block: say so once (an error here
    // surfaces at the launch)
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)batched_persistent, hipFuncAttributeMaxDynamicSharedMemorySize, kPersistSmem);
    (void)attr;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    hipLaunchKernelGGL(batched_persistent, dim3(cus * kPersistBlocksPerCU), dim3(256), kPersistSmem, st, a);
    return hipGetLastError();
}

}  // namespace psvt
