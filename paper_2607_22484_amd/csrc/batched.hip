// psvt_svt_batched / psvt_rank_r_batched: many soft-thresholdings of uneven
// shapes described by a DEVICE array of descriptors.  The host never sees
// the shapes: nothing is allocated, nothing is read back, every step is a
// kernel launch on the caller's stream, so the call can be captured into a
// HIP graph and replayed with new descriptor contents.
//
//   1. The host plans the method once for a template matrix (the planner of
//      the single calls, sentinel pointers, distinct sizes) and classifies
//      every matrix-dependent field of every stage (batched.h).  It checks
//      the classification by relocating the template to probe matrices of
//      both sides and comparing with their own plans, field for field.
//   2. A setup kernel reads the descriptors, checks them against the
//      maximum shape, lays out each valid matrix's workspace (layout.h,
//      prefix sum of the sizes), and for every count class (what a stage
//      launch enumerates: the tiles of one product kind in one tile
//      configuration, chosen per matrix by the same cost model as a single
//      call; norm partials; elementwise tiles) a prefix sum over matrices.
//   3. One launch per stage (products: one per tile configuration), each a
//      fixed grid that loops over its items; a block rebuilds each item's
//      descriptor from the stage template and the matrix record.
// Every tile is computed as in a single call, so results are bitwise the
// single calls'.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/psvt.h"
#include "batched.h"
#include "kernels.h"
#include "layout.h"
#include "plan.h"

using namespace psvt;

namespace psvt {
int plan_batched_matrix(int op, const psvt_batch_item &it, void *ws, const psvt_config *cfg, uint32_t *status,
                        std::vector<Stage> &out, Layout *layout);
int batched_cfg(const psvt_config *cfg, int *side, int *lp, int *persistent);
int set_error(int code, const char *msg);

static thread_local long long g_spin_limit = 1LL << 22;
void set_persist_spin_limit(long long polls) { g_spin_limit = polls; }
}  // namespace psvt

namespace {

constexpr int kMaxClasses = 48;
constexpr int64_t kMaxDim = 1 << 24;

// ------------------------------------------------------------ setup kernel

struct SetupArgs {
    const psvt_desc *descs;
    int count;
    int64_t max_m, max_n;
    int op, lp, side, status_on;
    char *area;          // per-matrix workspaces
    size_t area_bytes;
    MatInfo *mats;
    int *prefix;         // ncls x (count + 1)
    unsigned long long *need;  // count
    int ncls;
    CountClass cls[kMaxClasses];
    TileModelTable model;
};

__device__ inline bool desc_ok(const psvt_desc &d, const SetupArgs &a) {
    return d.A && d.Y && d.m >= 1 && d.n >= 1 && d.m <= a.max_m && d.n <= a.max_n && d.lda >= d.n &&
           d.ldy >= d.n && d.tau >= 0.0 && isfinite(d.tau);
}

// Exclusive prefix sum over the block (1024 threads, each a contiguous
// chunk), in a fixed order (deterministic); returns the total.
template <typename F>
__device__ unsigned long long block_scan(int count, F value, unsigned long long *out_each, int *out_int,
                                         unsigned long long *tmp) {
    const int T = blockDim.x, tid = threadIdx.x;
    const int chunk = (count + T - 1) / T;
    const int i0 = min(tid * chunk, count), i1 = min(i0 + chunk, count);
    unsigned long long sum = 0;
    for (int i = i0; i < i1; ++i) sum += value(i);
    tmp[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        unsigned long long run = 0;
        for (int k = 0; k < T; ++k) {
            const unsigned long long v = tmp[k];
            tmp[k] = run;
            run += v;
        }
        tmp[T] = run;
    }
    __syncthreads();
    unsigned long long run = tmp[tid];
    for (int i = i0; i < i1; ++i) {
        const unsigned long long v = value(i);  // before out_each[i] is written (it may be the input)
        if (out_each) out_each[i] = run;
        if (out_int) out_int[i] = (int)run;
        run += v;
    }
    const unsigned long long total = tmp[T];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(1024) void batched_setup(SetupArgs a) {
    __shared__ unsigned long long tmp[1025];
    for (int i = threadIdx.x; i < a.count; i += blockDim.x) {
        const psvt_desc d = a.descs[i];
        MatInfo mi;
        mi.A = d.A;
        mi.Y = d.Y;
        mi.status = a.status_on ? d.status : nullptr;
        mi.m = d.m;
        mi.n = d.n;
        mi.lda = d.lda;
        mi.ldy = d.ldy;
        mi.tau = d.tau;
        mi.valid = desc_ok(d, a) ? 1 : 0;
        mi.right = a.side == 1 ? 1 : a.side == 2 ? 0 : (d.n < d.m ? 1 : 0);
        mi.l = mi.right ? d.m : d.n;
        mi.s = mi.right ? d.n : d.m;
        mi.base = nullptr;
        a.need[i] = mi.valid ? (unsigned long long)layout_for(a.op, mi.l, mi.s, mi.right, a.lp, false).total : 0ull;
        a.mats[i] = mi;
    }
    __syncthreads();
    // workspace offsets; matrices beyond the area are skipped
    block_scan(a.count, [&](int i) { return a.need[i]; }, a.need, nullptr, tmp);
    for (int i = threadIdx.x; i < a.count; i += blockDim.x) {
        MatInfo &mi = a.mats[i];
        if (mi.valid) {
            const unsigned long long off = a.need[i];
            const unsigned long long sz = layout_for(a.op, mi.l, mi.s, mi.right, a.lp, false).total;
            if (off + sz > a.area_bytes) mi.valid = 0;
            else mi.base = a.area + off;
        }
        if (!mi.valid && a.status_on && a.descs[i].status) *a.descs[i].status = PSVT_STATUS_INVALID;
    }
    __syncthreads();
    for (int c = 0; c < a.ncls; ++c) {
        int *pre = a.prefix + (size_t)c * (a.count + 1);
        const CountClass cc = a.cls[c];
        const unsigned long long total =
            block_scan(a.count, [&](int i) { return (unsigned long long)class_count(cc, a.mats[i], a.model); },
                       nullptr, pre, tmp);
        if (threadIdx.x == 0) pre[a.count] = (int)total;
        __syncthreads();
    }
}

// --------------------------------------------------------- classification

// Template and probe matrices: sentinel pointers (16-byte aligned, never
// dereferenced) and sizes chosen so that every size and stride differs.
struct Sentinels {
    const float *A;
    float *Y;
    uint32_t *status;
    char *ws;
};
Sentinels sentinels(int k) {
    const uintptr_t base = (uintptr_t)0x7a0000000000ull + (uintptr_t)k * 0x1000000000ull;
    return Sentinels{(const float *)(base), (float *)(base + 0x100000000ull), (uint32_t *)(base + 0x200000000ull),
                     (char *)(base + 0x300000000ull)};
}

struct Template {
    int op, lp, side, persistent;
    std::vector<int> kind, dtype;
    std::vector<GemmStageT> g;
    std::vector<NormStageT> n;
    std::vector<TileStageT> t;
};

struct Classifier {
    Sentinels S;
    Layout L;
    int64_t m, n;
    bool ok = true;
    const char *why = "";

    uint8_t ptr(const void *p) {
        if (!p) return PC_NULL;
        if (p == (const void *)S.A) return PC_A;
        if (p == (const void *)S.Y) return PC_Y;
        if (p == (const void *)S.status) return PC_STATUS;
        const char *c = (const char *)p;
        if (c >= S.ws && c < S.ws + L.total) {
            const size_t off = (size_t)(c - S.ws);
            for (int b = 0; b < B_COUNT; ++b)
                if (L.has(b) && L.offset(b) == off) return (uint8_t)(PC_BUF + b);
        }
        ok = false;
        why = "a stage pointer that is no buffer, input or output";
        return PC_NULL;
    }
    uint8_t dim(int64_t v, bool io) {
        if (io) return v == m ? DC_M : v == n ? DC_N : DC_LIT;
        return v == L.l ? DC_L : v == L.s ? DC_S : DC_LIT;
    }
    uint8_t plane(int64_t v, uint8_t pcode) {
        return (pcode >= PC_BUF && v != 0 && v == L.plane(pcode - PC_BUF)) ? PL_BUF : PL_LIT;
    }
};

MatInfo probe_info(const Sentinels &S, int64_t m, int64_t n, int64_t lda, int64_t ldy, double tau, int side) {
    MatInfo mi;
    memset(&mi, 0, sizeof mi);
    mi.A = S.A;
    mi.Y = S.Y;
    mi.status = S.status;
    mi.m = m;
    mi.n = n;
    mi.lda = lda;
    mi.ldy = ldy;
    mi.tau = tau;
    mi.right = side == PSVT_SIDE_RIGHT ? 1 : side == PSVT_SIDE_LEFT ? 0 : (n < m ? 1 : 0);
    mi.l = mi.right ? m : n;
    mi.s = mi.right ? n : m;
    mi.base = S.ws;
    mi.valid = 1;
    return mi;
}

int plan_probe(int op, const MatInfo &mi, const psvt_config *cfg, std::vector<Stage> &out, Layout *L) {
    psvt_batch_item it;
    it.A = mi.A;
    it.Y = mi.Y;
    it.m = mi.m;
    it.n = mi.n;
    it.lda = mi.lda;
    it.ldy = mi.ldy;
    it.tau = mi.tau;
    return plan_batched_matrix(op, it, mi.base, cfg, mi.status, out, L);
}

// Plan the template matrix, classify its fields, and check the
// classification on probes of both sides.
int build_template(int op, const psvt_config *cfg, Template &T) {
    int rc = batched_cfg(cfg, &T.side, &T.lp, &T.persistent);
    if (rc) return rc;
    T.op = op;
    // template: a right-sided 333 x 201 matrix (unless the side is forced left)
    const Sentinels S0 = sentinels(0);
    const int64_t tm = T.side == PSVT_SIDE_LEFT ? 201 : 333, tn = T.side == PSVT_SIDE_LEFT ? 333 : 201;
    const MatInfo t0 = probe_info(S0, tm, tn, 1000, 1200, 0.3125, T.side);
    std::vector<Stage> st;
    Classifier C;
    C.S = S0;
    C.m = tm;
    C.n = tn;
    if ((rc = plan_probe(op, t0, cfg, st, &C.L))) return rc;
    for (const Stage &s : st) {
        T.kind.push_back(s.kind);
        T.dtype.push_back(s.dtype);
        GemmStageT g;
        NormStageT nn;
        TileStageT tt;
        memset(&g, 0, sizeof g);
        memset(&nn, 0, sizeof nn);
        memset(&tt, 0, sizeof tt);
        if (s.kind == ST_GEMM) {
            g.g = s.g;
            g.dtype = s.dtype;
            const void *ptrs[8] = {s.g.A, s.g.A2, s.g.B, s.g.D, s.g.C, s.g.CT, s.g.Clp, s.g.CTlp};
            for (int k = 0; k < 8; ++k) g.r.p[k] = C.ptr(ptrs[k]);
            g.r.pl[0] = C.plane(s.g.a_plane, g.r.p[0]);
            g.r.pl[1] = C.plane(s.g.b_plane, g.r.p[2]);
            g.r.pl[2] = C.plane(s.g.lp_plane, g.r.p[6]);
            g.r.pl[3] = C.plane(s.g.lp_plane_t, g.r.p[7]);
            g.r.M = C.dim(s.g.M, false);
            g.r.N = C.dim(s.g.N, false);
            g.r.K = C.dim(s.g.K, false);
            g.r.wa2_tau = s.g.A2 != nullptr;
            g.r.sc = s.g.sc != nullptr;
            g.r.swap_y = g.r.p[4] == PC_Y || g.r.p[5] == PC_Y;
            g.r.right_t = (uint8_t)t0.right;
        } else if (s.kind == ST_NORM) {
            nn.n = s.n;
            nn.r.X = C.ptr(s.n.X);
            const bool io = nn.r.X == PC_A || nn.r.X == PC_Y;
            nn.r.rows = C.dim(s.n.rows, io);
            nn.r.cols = C.dim(s.n.cols, io);
            nn.r.part = s.n.part != nullptr;
            nn.r.sc = s.n.sc != nullptr;
            nn.r.status = s.n.status != nullptr;
            nn.r.tau = s.n.mode == NORM_INPUT;
        } else {
            tt.t = s.t;
            tt.r.X = C.ptr(s.t.X);
            tt.r.Y = C.ptr(s.t.Y);
            tt.r.YT = C.ptr(s.t.YT);
            tt.r.L = C.ptr(s.t.L);
            const bool io = tt.r.X == PC_A;
            tt.r.rows = C.dim(s.t.rows, io);
            tt.r.cols = C.dim(s.t.cols, io);
            tt.r.lplane = C.plane(s.t.lplane, tt.r.L);
            tt.r.sc = s.t.sc != nullptr;
            tt.r.swap_t = s.t.kind == TOP_SCALE_T && io;
            tt.r.right_t = (uint8_t)t0.right;
        }
        T.g.push_back(g);
        T.n.push_back(nn);
        T.t.push_back(tt);
    }
    if (!C.ok) return set_error(PSVT_EINVAL, C.why);
    // probes: the template itself, a left-sided and a right-sided matrix of
    // other sizes, strides and thresholds
    struct P {
        int64_t m, n, lda, ldy;
        double tau;
    } probes[3] = {{tm, tn, 1000, 1200, 0.3125}, {150, 260, 300, 400, 0.75}, {97, 33, 40, 36, 1.5}};
    for (int k = 0; k < 3; ++k) {
        const MatInfo mi = probe_info(sentinels(k + 1), probes[k].m, probes[k].n, probes[k].lda, probes[k].ldy,
                                      probes[k].tau, T.side);
        std::vector<Stage> ps;
        if ((rc = plan_probe(op, mi, cfg, ps, nullptr))) return rc;
        if (ps.size() != st.size()) return set_error(PSVT_EINVAL, "internal: batched template has another stage count");
        for (size_t i = 0; i < ps.size(); ++i) {
            // first differing byte of the relocated template and the probe's own stage
            auto diff = [](const void *a, const void *b, size_t n) {
                for (size_t k = 0; k < n; ++k)
                    if (((const unsigned char *)a)[k] != ((const unsigned char *)b)[k]) return (long)k;
                return -1L;
            };
            long at = ps[i].kind == T.kind[i] ? -1 : 0;
            if (at < 0 && ps[i].kind == ST_GEMM) {
                GemmArgs g;
                relocate_gemm(T.g[i], mi, op, T.lp, g);
                at = ps[i].dtype != T.dtype[i] ? 0 : diff(&g, &ps[i].g, sizeof g);
            } else if (at < 0 && ps[i].kind == ST_NORM) {
                NormOp nn;
                relocate_norm(T.n[i], mi, op, T.lp, nn);
                at = diff(&nn, &ps[i].n, sizeof nn);
            } else if (at < 0) {
                TileOp tt;
                relocate_tile(T.t[i], mi, op, T.lp, tt);
                at = diff(&tt, &ps[i].t, sizeof tt);
            }
            if (at >= 0) {
                char msg[160];
                snprintf(msg, sizeof msg, "internal: batched stage %zu (%s, probe %d) does not relocate (byte %ld)", i,
                         ps[i].what ? ps[i].what : "?", k, at);
                return set_error(PSVT_EINVAL, msg);
            }
        }
    }
    return PSVT_OK;
}

// Count classes of the template's launches and the launch list.
struct Launch {
    int stage, tile, cls, final_pass;
};
int build_launches(const Template &T, std::vector<CountClass> &cls, std::vector<Launch> &out) {
    std::map<std::tuple<int, int, int, int, int, int, int, int, int, int, int>, int> index;
    auto get = [&](const CountClass &c) {
        auto key = std::make_tuple(c.kind, c.dtype, c.sym, c.tile, (int)c.c0, (int)c.c1, (int)c.c2, c.lit0, c.lit1,
                                   c.lit2, c.group);
        auto it = index.find(key);
        if (it != index.end()) return it->second;
        cls.push_back(c);
        return index[key] = (int)cls.size() - 1;
    };
    for (size_t k = 0; k < T.kind.size(); ++k) {
        CountClass c;
        memset(&c, 0, sizeof c);
        c.group = 1;
        if (T.kind[k] == ST_GEMM) {
            const GemmStageT &g = T.g[k];
            c.kind = CK_GEMM;
            c.dtype = g.dtype;
            c.sym = g.g.sym;
            c.c0 = g.r.M;
            c.c1 = g.r.N;
            c.c2 = g.r.K;
            c.lit0 = g.g.M;
            c.lit1 = g.g.N;
            c.lit2 = g.g.K;
            // the persistent executor holds a smaller tile set (tilemodel.h)
            const int hi = T.persistent ? kPersistMaxTile[g.dtype] : kNumTiles;
            for (int tile = 1; tile <= hi; ++tile) {
                c.tile = tile;
                out.push_back(Launch{(int)k, tile, get(c), 0});
            }
        } else if (T.kind[k] == ST_NORM) {
            c.kind = CK_NORM;
            c.c0 = T.n[k].r.rows;
            c.lit0 = (int)T.n[k].n.rows;
            c.c1 = T.n[k].r.cols;
            c.lit1 = (int)T.n[k].n.cols;
            out.push_back(Launch{(int)k, 0, get(c), 0});
            out.push_back(Launch{(int)k, 0, -1, 1});
        } else {
            c.kind = CK_TILE;
            c.c0 = T.t[k].r.rows;
            c.c1 = T.t[k].r.cols;
            c.lit0 = (int)T.t[k].t.rows;
            c.lit1 = (int)T.t[k].t.cols;
            // the persistent executor takes several elementwise tiles per
            // item (one ticket and one pair of fences each)
            c.group = T.persistent ? kPersistTileGroup : 1;
            out.push_back(Launch{(int)k, c.group, get(c), 0});
        }
    }
    if ((int)cls.size() > kMaxClasses) return set_error(PSVT_EINVAL, "internal: too many count classes");
    return PSVT_OK;
}

std::vector<PLaunch> plaunches(const std::vector<Launch> &launches) {
    std::vector<PLaunch> pl(launches.size());
    for (size_t j = 0; j < launches.size(); ++j)
        pl[j] = PLaunch{launches[j].stage, (int16_t)launches[j].cls, (int8_t)launches[j].tile,
                        (int8_t)launches[j].final_pass};
    return pl;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: [persistent control | records | prefix sums | sizes | stage
// templates | launches | first tickets | dependency counts | done counts]
// then the matrices' workspaces.  The persistent areas are empty (nl = 0)
// for the per-stage form.
struct Areas {
    size_t ctl, mats, prefix, need, stages, launches, lbase, deps, done, area, total;
};
Areas areas(int32_t count, int ncls, size_t per_matrix, int nstages = 0, int nl = 0) {
    Areas a;
    size_t off = 0;
    a.ctl = off;
    off = align256(off + (nl ? sizeof(PersistCtl) : 0));
    a.mats = off;
    off = align256(off + sizeof(MatInfo) * (size_t)count);
    a.prefix = off;
    off = align256(off + sizeof(int) * (size_t)ncls * ((size_t)count + 1));
    a.need = off;
    off = align256(off + sizeof(unsigned long long) * (size_t)count);
    a.stages = off;
    off = align256(off + (nl ? sizeof(StageT) * (size_t)nstages : 0));
    a.launches = off;
    off = align256(off + sizeof(PLaunch) * (size_t)nl);
    a.lbase = off;
    off = align256(off + (nl ? sizeof(int) * ((size_t)nl + 1) : 0));
    a.deps = off;
    off = align256(off + sizeof(int) * (size_t)count * (size_t)nl);
    a.done = off;
    off = align256(off + (nl ? sizeof(int) * (size_t)count : 0));
    a.area = off;
    a.total = off + per_matrix * (size_t)count;
    return a;
}

int check_shape_args(int32_t count, int64_t max_m, int64_t max_n) {
    if (count < 0 || count > (1 << 20)) return set_error(PSVT_EINVAL, "count outside 0..2^20");
    if (max_m < 1 || max_n < 1 || max_m > kMaxDim || max_n > kMaxDim)
        return set_error(PSVT_EINVAL, "max_m / max_n outside 1..2^24");
    // every prefix sum (tiles of the smallest configuration) must fit an int
    const double tiles = (double)count * ((max_m + 63) / 64) * (double)((max_n + 63) / 64) *
                         ((std::max(max_m, max_n) + 63) / 64);
    if (tiles >= 2147483647.0) return set_error(PSVT_EINVAL, "batch too large for one call");
    return PSVT_OK;
}

size_t per_matrix_bytes(int op, int64_t max_m, int64_t max_n, int lp) {
    // the layout grows with both sides, and every valid matrix has
    // l <= max(max_m, max_n), s <= min(max_m, max_n)
    return layout_for(op, std::max(max_m, max_n), std::min(max_m, max_n), true, lp != 0, false).total;
}

// The persistent executor numbers every item of the batch with an int.
int check_persistent_size(int32_t count, int64_t max_m, int64_t max_n, int nl) {
    const int64_t big = std::max(max_m, max_n);
    const double per = (double)((big + 63) / 64) * (double)((big + 63) / 64) + NORM_PARTIALS;
    if ((double)count * nl * per >= 2147483647.0) return set_error(PSVT_EINVAL, "batch too large for the persistent executor");
    return PSVT_OK;
}

int batched_workspace(int op, int32_t count, int64_t max_m, int64_t max_n, const psvt_config *cfg, size_t *bytes) {
    int rc = check_shape_args(count, max_m, max_n);
    if (rc) return rc;
    int side, lp, persistent;
    if ((rc = batched_cfg(cfg, &side, &lp, &persistent))) return rc;
    if (!count) {
        *bytes = 0;
        return PSVT_OK;
    }
    int nstages = 0, nl = 0;
    if (persistent) {  // the tables' sizes come from the plan
        Template T;
        std::vector<CountClass> cls;
        std::vector<Launch> launches;
        if ((rc = build_template(op, cfg, T)) || (rc = build_launches(T, cls, launches))) return rc;
        nstages = (int)T.kind.size();
        nl = (int)launches.size();
        if ((rc = check_persistent_size(count, max_m, max_n, nl))) return rc;
    }
    *bytes = areas(count, kMaxClasses, per_matrix_bytes(op, max_m, max_n, lp), nstages, nl).total;
    return PSVT_OK;
}

int batched_run(int op, const psvt_desc *d_descs, int32_t count, int64_t max_m, int64_t max_n, void *ws,
                size_t ws_bytes, const psvt_config *cfg, void *stream) {
    int rc = check_shape_args(count, max_m, max_n);
    if (rc) return rc;
    Template T;
    if ((rc = build_template(op, cfg, T))) return rc;
    if (count == 0) return PSVT_OK;
    if (!d_descs) return set_error(PSVT_EINVAL, "d_descs is NULL");
    std::vector<CountClass> cls;
    std::vector<Launch> launches;
    if ((rc = build_launches(T, cls, launches))) return rc;
    const int nstages = T.persistent ? (int)T.kind.size() : 0, nl = T.persistent ? (int)launches.size() : 0;
    if (T.persistent && (rc = check_persistent_size(count, max_m, max_n, nl))) return rc;
    const Areas A = areas(count, kMaxClasses, per_matrix_bytes(op, max_m, max_n, T.lp), nstages, nl);
    if (!ws || ws_bytes < A.total)
        return set_error(PSVT_EWORKSPACE, "batched workspace missing or smaller than psvt_batched_workspace_bytes()");
    if (((uintptr_t)ws & 255) != 0) return set_error(PSVT_EINVAL, "workspace is not 256-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return set_error(PSVT_EUNSUPPORTED, "device is not gfx950");
    char *base = (char *)ws;
    SetupArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.descs = d_descs;
    sa.count = count;
    sa.max_m = max_m;
    sa.max_n = max_n;
    sa.op = op;
    sa.lp = T.lp;
    sa.side = T.side;
    sa.status_on = cfg && (cfg->flags & PSVT_FLAG_STATUS) ? 1 : 0;
    sa.area = base + A.area;
    sa.area_bytes = ws_bytes - A.area;
    sa.mats = (MatInfo *)(base + A.mats);
    sa.prefix = (int *)(base + A.prefix);
    sa.need = (unsigned long long *)(base + A.need);
    sa.ncls = (int)cls.size();
    for (size_t c = 0; c < cls.size(); ++c) sa.cls[c] = cls[c];
    sa.model = T.persistent ? tile_model_persistent() : tile_model();
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(batched_setup, dim3(1), dim3(1024), 0, st, sa);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
    if (T.persistent) {
        std::vector<StageT> stages(T.kind.size());
        for (size_t k = 0; k < T.kind.size(); ++k) {
            StageT &x = stages[k];
            memset(&x, 0, sizeof x);
            x.kind = T.kind[k];
            x.dtype = T.dtype[k];
            if (x.kind == ST_GEMM)
                x.g = T.g[k];
            else if (x.kind == ST_NORM)
                x.n = T.n[k];
            else
                x.t = T.t[k];
        }
        const std::vector<PLaunch> pl = plaunches(launches);
        if ((e = launch_upload(base + A.stages, stages.data(), sizeof(StageT) * stages.size(), st)) != hipSuccess ||
            (e = launch_upload(base + A.launches, pl.data(), sizeof(PLaunch) * pl.size(), st)) != hipSuccess)
            return set_error(PSVT_EHIP, hipGetErrorString(e));
        PersistArgs pa;
        memset(&pa, 0, sizeof pa);
        pa.mats = sa.mats;
        pa.count = count;
        pa.op = op;
        pa.lp = T.lp;
        pa.status_on = sa.status_on;
        pa.prefix = sa.prefix;
        pa.launches = (const PLaunch *)(base + A.launches);
        pa.nl = nl;
        pa.stages = (const StageT *)(base + A.stages);
        pa.lbase = (int *)(base + A.lbase);
        pa.deps = (int *)(base + A.deps);
        pa.done = (int *)(base + A.done);
        pa.ctl = (PersistCtl *)(base + A.ctl);
        pa.spin_limit = g_spin_limit;
        if ((e = launch_persistent(pa, st)) != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
        return PSVT_OK;
    }
    BatchView v;
    v.mats = sa.mats;
    v.count = count;
    v.op = op;
    v.lp = T.lp;
    for (const Launch &L : launches) {
        v.prefix = L.cls >= 0 ? sa.prefix + (size_t)L.cls * ((size_t)count + 1) : sa.prefix;
        const int k = L.stage;
        if (T.kind[k] == ST_GEMM)
            e = launch_gemm_batched(v, T.g[k], L.tile, st);
        else if (T.kind[k] == ST_NORM)
            e = launch_norm_batched(v, T.n[k], L.final_pass, st);
        else
            e = launch_tile_batched(v, T.t[k], st);
        if (e != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
    }
    return PSVT_OK;
}

// Host replay of the persistent executor's schedule for the given shapes:
// the records, count classes and tables the setup kernels would build (the
// same functions), then checks that tickets map one to one onto items in
// (launch, matrix, item) order, that an item's dependency count is the
// matrix's items of earlier launches, and that `blocks` simulated blocks
// taking tickets in order, with random item durations, drain every ticket,
// each item starting only after its matrix's earlier launches completed.
int check_schedule(int op, const int64_t *ms, const int64_t *ns, int32_t count, int64_t max_m, int64_t max_n,
                   const psvt_config *cfg, int32_t blocks, uint64_t seed, int64_t *tickets) {
    int rc = check_shape_args(count, max_m, max_n);
    if (rc) return rc;
    if (!ms || !ns || !tickets || blocks < 1) return set_error(PSVT_EINVAL, "bad arguments");
    Template T;
    if ((rc = build_template(op, cfg, T))) return rc;
    T.persistent = 1;
    std::vector<CountClass> cls;
    std::vector<Launch> launches;
    if ((rc = build_launches(T, cls, launches))) return rc;
    const std::vector<PLaunch> pl = plaunches(launches);
    const int nl = (int)pl.size();
    const TileModelTable model = tile_model_persistent();
    std::vector<MatInfo> mats(count);
    for (int i = 0; i < count; ++i) {
        MatInfo &mi = mats[i];
        memset(&mi, 0, sizeof mi);
        mi.m = ms[i];
        mi.n = ns[i];
        mi.valid = ms[i] >= 1 && ns[i] >= 1 && ms[i] <= max_m && ns[i] <= max_n;
        mi.right = T.side == PSVT_SIDE_RIGHT ? 1 : T.side == PSVT_SIDE_LEFT ? 0 : (ns[i] < ms[i] ? 1 : 0);
        mi.l = mi.right ? mi.m : mi.n;
        mi.s = mi.right ? mi.n : mi.m;
    }
    const size_t cs = (size_t)count + 1;
    std::vector<int> prefix(cls.size() * cs);
    for (size_t c = 0; c < cls.size(); ++c) {
        int run = 0;
        for (int i = 0; i < count; ++i) {
            prefix[c * cs + i] = run;
            run += class_count(cls[c], mats[i], model);
        }
        prefix[c * cs + count] = run;
    }
    for (int j = 0; j < nl; ++j)
        if (T.kind[pl[j].stage] == ST_GEMM && prefix[(size_t)pl[j].cls * cs + count] > 0 &&
            pl[j].tile > kPersistMaxTile[T.dtype[pl[j].stage]])
            return set_error(PSVT_EINVAL, "schedule: a launch outside the executor's tile set has items");
    std::vector<int> lbase(nl + 1), deps((size_t)count * nl);
    {
        int run = 0;
        for (int j = 0; j < nl; ++j) {
            lbase[j] = run;
            run += persist_launch_items(pl[j], prefix.data(), count);
        }
        lbase[nl] = run;
        for (int i = 0; i < count; ++i) {
            int r = 0;
            for (int j = 0; j < nl; ++j) {
                deps[(size_t)i * nl + j] = r;
                r += persist_items(pl[j], prefix.data(), count, i);
            }
        }
    }
    const int total = lbase[nl];
    // tickets in (launch, matrix, item) order
    {
        int t = 0;
        for (int j = 0; j < nl; ++j)
            for (int i = 0; i < count; ++i)
                for (int k = 0, n = persist_items(pl[j], prefix.data(), count, i); k < n; ++k, ++t) {
                    int dj, di, dk;
                    persist_decode(lbase.data(), nl, pl.data(), prefix.data(), count, t, dj, di, dk);
                    if (dj != j || di != i || dk != k) {
                        char msg[160];
                        snprintf(msg, sizeof msg, "schedule: ticket %d decodes to (%d, %d, %d), not (%d, %d, %d)", t,
                                 dj, di, dk, j, i, k);
                        return set_error(PSVT_EINVAL, msg);
                    }
                }
        if (t != total) return set_error(PSVT_EINVAL, "schedule: ticket count differs from the items");
    }
    // simulated blocks: take the next ticket when idle, wait for the
    // matrix's dependency count, run for a random time
    uint64_t x = seed * 2654435761ull + 0x9e3779b97f4a7c15ull;
    auto rnd = [&]() {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        return x;
    };
    struct Blk {
        int T, j, i;
        int state;  // 0 idle, 1 waiting, 2 running
        uint64_t end;
    };
    std::vector<Blk> b(blocks, Blk{-1, 0, 0, 0, 0});
    std::vector<int> done(count, 0);
    int next = 0, finished = 0;
    uint64_t now = 0;
    while (finished < total) {
        bool progress = false;
        for (Blk &k : b) {
            if (k.state == 0 && next < total) {
                k.T = next++;
                int item;
                persist_decode(lbase.data(), nl, pl.data(), prefix.data(), count, k.T, k.j, k.i, item);
                k.state = 1;
                progress = true;
            }
            if (k.state == 1) {
                const int want = deps[(size_t)k.i * nl + k.j];
                if (done[k.i] >= want) {
                    // nothing of a later launch of this matrix may have completed
                    if (done[k.i] >= want + persist_items(pl[k.j], prefix.data(), count, k.i))
                        return set_error(PSVT_EINVAL, "schedule: an item ran after a later one of its matrix");
                    k.state = 2;
                    k.end = now + 1 + rnd() % 1000;
                    progress = true;
                }
            }
        }
        int first = -1;
        for (int q = 0; q < blocks; ++q)
            if (b[q].state == 2 && (first < 0 || b[q].end < b[first].end)) first = q;
        if (first < 0) {
            if (!progress) return set_error(PSVT_EINVAL, "schedule: simulated blocks deadlock");
            continue;
        }
        now = b[first].end;
        ++done[b[first].i];
        ++finished;
        b[first].state = 0;
    }
    for (int i = 0; i < count; ++i)
        if (done[i] != (nl ? deps[(size_t)i * nl + nl - 1] + persist_items(pl[nl - 1], prefix.data(), count, i) : 0))
            return set_error(PSVT_EINVAL, "schedule: a matrix did not complete all its items");
    *tickets = total;
    return PSVT_OK;
}

}  // namespace

extern "C" {

int psvt_batched_check_schedule(int op, const int64_t *ms, const int64_t *ns, int32_t count, int64_t max_m,
                                int64_t max_n, const psvt_config *cfg, int32_t blocks, uint64_t seed,
                                int64_t *tickets) {
    if (op != PSVT_OP_SVT && op != PSVT_OP_RANK_R) return set_error(PSVT_EINVAL, "op must be svt or rank_r");
    return check_schedule(op, ms, ns, count, max_m, max_n, cfg, blocks, seed, tickets);
}


int psvt_batched_workspace_bytes(int op, int32_t count, int64_t max_m, int64_t max_n, const psvt_config *cfg,
                                 size_t *bytes) {
    if (!bytes) return set_error(PSVT_EINVAL, "bytes is NULL");
    if (op != PSVT_OP_SVT && op != PSVT_OP_RANK_R) return set_error(PSVT_EINVAL, "op must be svt or rank_r");
    return batched_workspace(op, count, max_m, max_n, cfg, bytes);
}

int psvt_svt_batched(const psvt_desc *d_descs, int32_t count, int64_t max_m, int64_t max_n, void *ws,
                     size_t ws_bytes, const psvt_config *cfg, void *stream) {
    return batched_run(PSVT_OP_SVT, d_descs, count, max_m, max_n, ws, ws_bytes, cfg, stream);
}

int psvt_rank_r_batched(const psvt_desc *d_descs, int32_t count, int64_t max_m, int64_t max_n, void *ws,
                        size_t ws_bytes, const psvt_config *cfg, void *stream) {
    return batched_run(PSVT_OP_RANK_R, d_descs, count, max_m, max_n, ws, ws_bytes, cfg, stream);
}

}  // extern "C"
