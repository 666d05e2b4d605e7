// Batched form: many soft-thresholdings of uneven shapes executed stage by
// stage with grouped launches, replayed as one HIP graph.
//
// Every matrix of a batch runs the same stage list (same iteration schedule),
// so stage k of all matrices is one launch per tile configuration:
//   - products: each matrix's tile configuration comes from the autotuned
//     cost model (its size class); products sharing a configuration go into
//     one grouped launch whose blocks find their product by binary search in
//     a prefix sum of tile counts, largest products first, so the hardware
//     dispatcher balances the uneven work;
//   - norms and tiled elementwise passes: one grouped launch each.
// The descriptor tables live in one device buffer written at creation; a
// run only enqueues kernels (no allocation, no host synchronisation), and the
// whole run is captured once into a graph.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/psvt.h"
#include "kernels.h"
#include "plan.h"

using namespace psvt;

namespace psvt {
// provided by api.hip
int batch_plan_one(int op, const psvt_batch_item &it, void *ws, const psvt_config *cfg, std::vector<Stage> &out,
                   size_t *ws_bytes);
int set_error(int code, const char *msg);
}  // namespace psvt

namespace {

struct Launch {
    int kind;  // ST_GEMM / ST_NORM / ST_TILE
    int dtype, tile, sym, two_a, tkind;
    size_t ops_off, prefix_off;
    int n, total;
    double flops, bytes;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct psvt_batch {
    int count = 0;
    std::vector<Launch> launches;
    std::vector<char> host;  // descriptor tables (uploaded to dev)
    char *dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace {

int enqueue(psvt_batch *b, hipStream_t st) {
    for (const Launch &L : b->launches) {
        hipError_t e = hipSuccess;
        if (L.kind == ST_GEMM)
            e = launch_gemm_grouped((const GemmArgs *)(b->dev + L.ops_off), (const int *)(b->dev + L.prefix_off), L.n,
                                    L.total, L.dtype, L.tile, L.sym, L.two_a, L.flops, st);
        else if (L.kind == ST_NORM)
            e = launch_norm_grouped((const NormOp *)(b->dev + L.ops_off), (const int *)(b->dev + L.prefix_off), L.n,
                                    L.total, L.bytes, st);
        else
            e = launch_tile_op_grouped((const TileOp *)(b->dev + L.ops_off), (const int *)(b->dev + L.prefix_off),
                                       L.n, L.total, L.tkind, L.bytes, st);
        if (e != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
    }
    return PSVT_OK;
}

template <typename T>
size_t push_table(std::vector<char> &host, const std::vector<T> &v) {
    size_t off = align_up(host.size(), 256);
    host.resize(off + sizeof(T) * v.size());
    memcpy(host.data() + off, v.data(), sizeof(T) * v.size());
    return off;
}

// Stage k of every plan -> grouped launches.
int build_stage(psvt_batch *b, const std::vector<std::vector<Stage>> &plans, size_t k) {
    const Stage &s0 = plans[0][k];
    for (const auto &p : plans)
        if (p[k].kind != s0.kind || (s0.kind == ST_GEMM && (p[k].dtype != s0.dtype || p[k].g.sym != s0.g.sym ||
                                                             (p[k].g.A2 != nullptr) != (s0.g.A2 != nullptr))) ||
            (s0.kind == ST_TILE && p[k].t.kind != s0.t.kind))
            return set_error(PSVT_EINVAL, "batch items do not share a stage structure");
    const int n = (int)plans.size();
    if (s0.kind == ST_GEMM) {
        // group by tile configuration, largest modelled time first
        std::vector<int> tile(n);
        std::vector<double> cost(n);
        for (int i = 0; i < n; ++i) {
            tile[i] = gemm_pick_tile(plans[i][k].g, s0.dtype);
            cost[i] = gemm_model_us(plans[i][k].g, s0.dtype, tile[i]);
        }
        for (int t = 1; t <= 4; ++t) {
            std::vector<int> idx;
            for (int i = 0; i < n; ++i)
                if (tile[i] == t) idx.push_back(i);
            if (idx.empty()) continue;
            std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost[x] > cost[y]; });
            std::vector<GemmArgs> args;
            std::vector<int> prefix;
            int total = 0;
            double flops = 0.0;
            for (int i : idx) {
                const GemmArgs &g = plans[i][k].g;
                args.push_back(g);
                prefix.push_back(total);
                total += gemm_tile_count(g, t);
                flops += g.sym ? (double)g.M * (g.M + 1) * g.K : 2.0 * g.M * g.N * g.K;
            }
            Launch L{};
            L.kind = ST_GEMM;
            L.dtype = s0.dtype;
            L.tile = t;
            L.sym = s0.g.sym;
            L.two_a = s0.g.A2 != nullptr;
            L.n = (int)idx.size();
            L.total = total;
            L.flops = flops;
            L.ops_off = push_table(b->host, args);
            L.prefix_off = push_table(b->host, prefix);
            b->launches.push_back(L);
        }
    } else if (s0.kind == ST_NORM) {
        std::vector<NormOp> ops;
        std::vector<int> prefix;
        int total = 0;
        double bytes = 0.0;
        for (int i = 0; i < n; ++i) {
            ops.push_back(plans[i][k].n);
            prefix.push_back(total);
            total += plans[i][k].n.nparts;
            bytes += 4.0 * plans[i][k].n.rows * plans[i][k].n.cols;
        }
        Launch L{};
        L.kind = ST_NORM;
        L.n = n;
        L.total = total;
        L.bytes = bytes;
        L.ops_off = push_table(b->host, ops);
        L.prefix_off = push_table(b->host, prefix);
        b->launches.push_back(L);
    } else {
        std::vector<TileOp> ops;
        std::vector<int> prefix;
        int total = 0;
        double bytes = 0.0;
        for (int i = 0; i < n; ++i) {
            ops.push_back(plans[i][k].t);
            prefix.push_back(total);
            total += tile_op_tiles(plans[i][k].t);
            bytes += tile_op_bytes(plans[i][k].t);
        }
        Launch L{};
        L.kind = ST_TILE;
        L.tkind = s0.t.kind;
        L.n = n;
        L.total = total;
        L.bytes = bytes;
        L.ops_off = push_table(b->host, ops);
        L.prefix_off = push_table(b->host, prefix);
        b->launches.push_back(L);
    }
    return PSVT_OK;
}

int check_items(int op, const psvt_batch_item *items, int32_t count) {
    if (op != PSVT_OP_SVT && op != PSVT_OP_RANK_R) return set_error(PSVT_EINVAL, "batched op must be svt or rank_r");
    if (!items || count <= 0) return set_error(PSVT_EINVAL, "no batch items");
    for (int i = 0; i < count; ++i) {
        const psvt_batch_item &it = items[i];
        if (it.m < 1 || it.n < 1 || it.m > (1 << 20) || it.n > (1 << 20))
            return set_error(PSVT_EINVAL, "batch item with a bad size");
        if (!it.A || !it.Y || it.lda < it.n || it.ldy < it.n)
            return set_error(PSVT_EINVAL, "batch item with a NULL pointer or bad leading dimension");
        if (!(it.tau >= 0.0) || it.tau > 1e300) return set_error(PSVT_EINVAL, "batch item with a bad tau");
    }
    return PSVT_OK;
}

}  // namespace

extern "C" {

int psvt_batch_workspace_bytes(int op, const psvt_batch_item *items, int32_t count, const psvt_config *cfg,
                               size_t *bytes) {
    int rc = check_items(op, items, count);
    if (rc) return rc;
    if (!bytes) return set_error(PSVT_EINVAL, "bytes is NULL");
    size_t total = 0;
    for (int i = 0; i < count; ++i) {
        std::vector<Stage> tmp;
        size_t one = 0;
        if ((rc = batch_plan_one(op, items[i], nullptr, cfg, tmp, &one))) return rc;
        total = align_up(total, 256) + one;
    }
    *bytes = total;
    return PSVT_OK;
}

int psvt_batch_create(int op, const psvt_batch_item *items, int32_t count, void *ws, size_t ws_bytes,
                      const psvt_config *cfg, psvt_batch **out) {
    if (!out) return set_error(PSVT_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_items(op, items, count);
    if (rc) return rc;
    if (!ws || ((uintptr_t)ws & 255)) return set_error(PSVT_EWORKSPACE, "workspace NULL or not 256-byte aligned");
    std::vector<std::vector<Stage>> plans(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        off = align_up(off, 256);
        size_t one = 0;
        if ((rc = batch_plan_one(op, items[i], (char *)ws + off, cfg, plans[i], &one))) return rc;
        off += one;
        if (off > ws_bytes) return set_error(PSVT_EWORKSPACE, "batch workspace too small");
        if (plans[i].size() != plans[0].size()) return set_error(PSVT_EINVAL, "batch items differ in stage count");
    }
    psvt_batch *b = new psvt_batch();
    b->count = count;
    for (size_t k = 0; k < plans[0].size(); ++k)
        if ((rc = build_stage(b, plans, k))) {
            delete b;
            return rc;
        }
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc((void **)&b->dev, std::max<size_t>(b->host.size(), 256));
    if (e == hipSuccess) e = hipMemcpy(b->dev, b->host.data(), b->host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (b->dev) (void)hipFree(b->dev);
        delete b;
        return set_error(PSVT_EHIP, hipGetErrorString(e));
    }
    // capture one run into a graph
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue(b, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (rc == PSVT_OK && e2 == hipSuccess) {
            b->graph = g;
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        } else {
            if (g) (void)hipGraphDestroy(g);
            e = e2 != hipSuccess ? e2 : hipErrorUnknown;
        }
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        psvt_batch_destroy(b);
        return set_error(PSVT_EHIP, hipGetErrorString(e));
    }
    *out = b;
    return PSVT_OK;
}

int psvt_batch_run(psvt_batch *b, void *stream) {
    if (!b) return set_error(PSVT_EINVAL, "batch is NULL");
    return enqueue(b, (hipStream_t)stream);
}

int psvt_batch_run_graph(psvt_batch *b, void *stream) {
    if (!b || !b->exec) return set_error(PSVT_EINVAL, "batch is NULL or has no graph");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
    return PSVT_OK;
}

int psvt_batch_stats(const psvt_batch *b, int32_t *launches, double *flops) {
    if (!b) return set_error(PSVT_EINVAL, "batch is NULL");
    double f = 0.0;
    for (const Launch &L : b->launches) f += L.flops;
    if (launches) *launches = (int32_t)b->launches.size();
    if (flops) *flops = f;
    return PSVT_OK;
}

int psvt_batch_destroy(psvt_batch *b) {
    if (!b) return PSVT_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->dev) (void)hipFree(b->dev);
    delete b;
    return PSVT_OK;
}

}  // extern "C"
