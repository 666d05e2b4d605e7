// Serving core: a request loop for soft-thresholding calls of mixed sizes,
// with admission by an HBM budget and iteration-level continuous batching.
//
// Requests are admitted in arrival order while a slot is free and the
// server's device memory pool (the HBM budget) has room for the request's
// workspace; their iterates then live in that workspace until completion.
// A worker thread runs ticks.  In one tick every active request advances
// by up to `rounds` stages of its stage list; the stages of one round are
// grouped by kind (products also by operand type and tile configuration)
// into grouped launches, so requests at different points of their iteration
// share launches and a request admitted during the run joins at the next
// tick.  Requests are split by size into lanes; each lane runs its own ticks
// on its own stream, so lanes overlap on the device and small requests do
// not advance at the pace of the largest stages.  Each product tile is computed exactly as in a single call, so a
// result does not depend on what it was batched with.  At most `depth` + 1
// ticks of a lane are in flight on its stream; a request completes when the
// event of the tick that launched its last stage has passed, and its
// workspace returns to the pool.
//
// With PSVT_SERVER_FAKE the same scheduler runs without a device: stages
// complete immediately (for testing admission and scheduling on a CPU).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/psvt.h"
#include "kernels.h"
#include "plan.h"

using namespace psvt;

namespace psvt {
int plan_request(int op, const psvt_batch_item &it, void *ws, const psvt_config *cfg, std::vector<Stage> &out,
                 size_t *ws_bytes, bool check_dev, size_t *chains);
int set_error(int code, const char *msg);
}  // namespace psvt

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) in 256-byte units.
class Pool {
  public:
    explicit Pool(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(std::max<size_t>(bytes, 256));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(std::max<size_t>(bytes, 256));
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
    size_t used_ = 0, peak_ = 0;
};

enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2, RQ_FAILED = -1 };

struct Request {
    uint64_t ticket;
    int op;
    psvt_batch_item item;
    size_t ws_bytes = 0, ws_off = 0;
    std::vector<Stage> plan;
    // plan[0, cut[0]) common prefix, [cut[0], cut[1]) P iterations, [cut[1],
    // cut[2]) S iterations, then the final product; the two iteration chains
    // advance independently (a round takes the next stage of each)
    size_t cut[3] = {0, 0, 0};
    size_t cursor = 0, curP = 0, curS = 0;
    int state = RQ_QUEUED;
    // recorded on the submitter's stream at submit: the request's first
    // stage waits for it, so A and Y are ordered after the caller's work
    hipEvent_t ready = nullptr;
    bool waited = false;       // the lane stream already waits for `ready`
    bool parked = false;       // admitted, waiting for the lane's next cohort
    int64_t finish_tick = -1;  // lane tick that launched the last stage
    int lane = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

// Stages a request can run next (at most two: one of each iteration chain).
int next_stages(const Request *r, size_t idx[2]) {
    if (r->cursor < r->cut[0]) {
        idx[0] = r->cursor;
        return 1;
    }
    int n = 0;
    if (r->curP < r->cut[1]) idx[n++] = r->curP;
    if (r->curS < r->cut[2]) idx[n++] = r->curS;
    if (n) return n;
    const size_t f = std::max(r->cursor, r->cut[2]);
    if (f < r->plan.size()) {
        idx[0] = f;
        return 1;
    }
    return 0;
}

bool plan_done(const Request *r) {
    size_t idx[2];
    return next_stages(r, idx) == 0;
}

void advance(Request *r, size_t i) {
    if (i < r->cut[0] || i >= r->cut[2])
        r->cursor = i + 1;
    else if (i < r->cut[1])
        r->curP = i + 1;
    else
        r->curS = i + 1;
}

// Lane of a request: by s^2 l (s, l the short and long side), the scale of
// its flops, in factors of 8 from 512^3.
int lane_of(const psvt_batch_item &it, int nlanes) {
    const double s = (double)std::min(it.m, it.n), l = (double)std::max(it.m, it.n);
    const double w = s * s * l;
    int lane = 0;
    for (double t = 512.0 * 512.0 * 512.0; lane < nlanes - 1 && w > t; t *= 8.0) ++lane;
    return lane;
}

}  // namespace

struct psvt_server {
    bool fake = false;
    bool cohort = false;  // lanes start admitted requests in cohorts
    size_t budget = 0;
    int max_slots = 1, rounds = 3, depth = 3;
    psvt_config cfg{};
    std::vector<double> coeffs;
    char *pool_dev = nullptr;
    Pool *pool = nullptr;
    int device = 0;

    // Lanes: requests are assigned by size (s^2 l, the flop scale) to one of
    // kLanes lanes; a lane runs its own ticks on its own stream, so small
    // requests do not advance at the pace of the largest stages, and the
    // lanes' launches overlap on the device.  Each lane has a descriptor ring
    // of one 1 MiB segment per in-flight tick.
    static constexpr size_t kSegBytes = 1 << 20;
    static constexpr int kLanes = 4;
    struct Lane {
        hipStream_t stream = nullptr;
        std::vector<hipEvent_t> seg_event;
        std::vector<int64_t> seg_tick;
        int64_t tick = 0;
        size_t rr = 0;  // rotation of the runnable list when a tick cannot take them all
        char *ring_host = nullptr, *ring_dev = nullptr;
    };
    Lane lanes[kLanes];
    int nseg = 0;
    char *ring_host = nullptr, *ring_dev = nullptr;  // all lanes' segments

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    int error = PSVT_OK;
    std::vector<hipEvent_t> free_events;  // ready events of finished requests

    // request deadline (seconds from submit; 0 = none) and the workspaces of
    // failed requests that the lane's in-flight ticks may still use
    double timeout_s = 0.0;
    struct Pending {
        int lane;
        int64_t tick;
        size_t off, bytes;
    };
    std::vector<Pending> pending;
    // fault injection (fake servers: tests of the failure paths)
    int64_t fault_tick = -1, fault_plan = -1, plans = 0;
    bool stall = false;

    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, timed_out = 0, ticks = 0, launches = 0;
    std::vector<double> latency_ms, queue_ms;
    double first_submit = -1, last_done = -1;
};

namespace {

// Grouped launches of one round (stages with equal signatures).
struct GroupKey {
    int kind, dtype, sym, two_a, tile, tkind;
    bool operator<(const GroupKey &o) const {
        return std::tie(kind, dtype, sym, two_a, tile, tkind) < std::tie(o.kind, o.dtype, o.sym, o.two_a, o.tile, o.tkind);
    }
};

// One grouped launch of a round: descriptors at `off` in the segment, the
// tile prefix after them.
struct Group {
    GroupKey k;
    size_t off;
    int n, total;
    double flops, bytes;
};

// Host side of one round: the groups' descriptors into the segment (after
// seg_used), the requests' cursors advanced; the launches are appended to gl.
int build_round(psvt_server *s, psvt_server::Lane &lane, std::vector<Request *> &reqs, int seg, size_t &seg_used,
                std::vector<Group> &gl) {
    typedef std::pair<Request *, size_t> Entry;  // (request, stage index)
    std::map<GroupKey, std::vector<Entry>> groups;
    std::vector<Entry> taken;
    for (Request *r : reqs) {
        size_t idx[2];
        const int n = next_stages(r, idx);
        for (int e = 0; e < n; ++e) {
            const Stage &st = r->plan[idx[e]];
            GroupKey k{st.kind, st.kind == ST_GEMM ? st.dtype : 0, st.kind == ST_GEMM ? st.g.sym : 0,
                       st.kind == ST_GEMM ? (st.g.A2 != nullptr) : 0,
                       st.kind == ST_GEMM ? gemm_pick_tile(st.g, st.dtype) : 0, st.kind == ST_TILE ? st.t.kind : 0};
            groups[k].push_back(Entry(r, idx[e]));
            taken.push_back(Entry(r, idx[e]));
        }
    }
    char *hseg = lane.ring_host + (size_t)seg * psvt_server::kSegBytes;
    const size_t first = gl.size();
    // every group's descriptors into this round's part of the segment
    for (auto &kv : groups) {
        const GroupKey &k = kv.first;
        auto &rs = kv.second;
        if (k.kind == ST_GEMM)  // largest first
            std::stable_sort(rs.begin(), rs.end(), [&](const Entry &a, const Entry &b) {
                return gemm_model_us(a.first->plan[a.second].g, k.dtype, k.tile) >
                       gemm_model_us(b.first->plan[b.second].g, k.dtype, k.tile);
            });
        const size_t esz = k.kind == ST_GEMM ? sizeof(GemmArgs) : (k.kind == ST_NORM ? sizeof(NormOp) : sizeof(TileOp));
        const size_t need = align256(esz * rs.size()) + align256(sizeof(int) * rs.size());
        if (seg_used + need > psvt_server::kSegBytes) return set_error(PSVT_EINVAL, "server descriptor segment full");
        char *hops = hseg + seg_used, *hpre = hops + align256(esz * rs.size());
        Group G{k, seg_used, (int)rs.size(), 0, 0.0, 0.0};
        for (size_t i = 0; i < rs.size(); ++i) {
            const Stage &st = rs[i].first->plan[rs[i].second];
            ((int *)hpre)[i] = G.total;
            if (k.kind == ST_GEMM) {
                ((GemmArgs *)hops)[i] = st.g;
                G.total += gemm_tile_count(st.g, k.tile);
                G.flops += st.g.sym ? (double)st.g.M * (st.g.M + 1) * st.g.K : 2.0 * st.g.M * st.g.N * st.g.K;
            } else if (k.kind == ST_NORM) {
                ((NormOp *)hops)[i] = st.n;
                G.total += st.n.nparts;
                G.bytes += 4.0 * st.n.rows * st.n.cols;
            } else {
                ((TileOp *)hops)[i] = st.t;
                G.total += tile_op_tiles(st.t);
                G.bytes += tile_op_bytes(st.t);
            }
        }
        seg_used += need;
        gl.push_back(G);
    }
    s->launches += (int64_t)(gl.size() - first);
    for (const Entry &e : taken) advance(e.first, e.second);
    return PSVT_OK;
}

// Device side of one tick: one descriptor copy for all its rounds, then the
// rounds' launches in order on the lane's stream.
int launch_tick(psvt_server *s, psvt_server::Lane &lane, int seg, size_t seg_used, const std::vector<Group> &gl) {
    if (s->fake || gl.empty()) return PSVT_OK;
    char *hseg = lane.ring_host + (size_t)seg * psvt_server::kSegBytes;
    char *dseg = lane.ring_dev + (size_t)seg * psvt_server::kSegBytes;
    hipError_t e = hipMemcpyAsync(dseg, hseg, seg_used, hipMemcpyHostToDevice, lane.stream);
    for (size_t gi = 0; gi < gl.size() && e == hipSuccess; ++gi) {
        const Group &G = gl[gi];
        const GroupKey &k = G.k;
        const size_t esz = k.kind == ST_GEMM ? sizeof(GemmArgs) : (k.kind == ST_NORM ? sizeof(NormOp) : sizeof(TileOp));
        const char *dops = dseg + G.off, *dpre = dops + align256(esz * G.n);
        if (k.kind == ST_GEMM)
            e = launch_gemm_grouped((const GemmArgs *)dops, (const int *)dpre, G.n, G.total, k.dtype, k.tile, k.sym,
                                    k.two_a, G.flops, lane.stream);
        else if (k.kind == ST_NORM)
            e = launch_norm_grouped((const NormOp *)dops, (const int *)dpre, G.n, G.total, G.bytes, lane.stream);
        else
            e = launch_tile_op_grouped((const TileOp *)dops, (const int *)dpre, G.n, G.total, k.tkind, G.bytes,
                                       lane.stream);
    }
    if (e != hipSuccess) return set_error(PSVT_EHIP, hipGetErrorString(e));
    return PSVT_OK;
}

// Whether lane tick `tick` has finished on the device (fake: at once).
bool tick_passed(psvt_server *s, int lane, int64_t tick) {
    if (s->fake || tick < 0) return true;
    const psvt_server::Lane &ln = s->lanes[lane];
    const int seg = (int)(tick % s->nseg);
    return ln.seg_tick[seg] != tick || hipEventQuery(ln.seg_event[seg]) == hipSuccess;
}

// keep_ws: the request's stages may still be in flight on its lane; its
// workspace returns to the pool once the lane's latest tick has passed.
void finish(psvt_server *s, Request *r, int state, bool keep_ws = false) {
    r->state = state;
    r->t_done = now_s();
    if (r->ready) {  // the lane waited for it before the request's first stage (or never will)
        if (!keep_ws) s->free_events.push_back(r->ready);  // else an in-flight wait may still name it
        r->ready = nullptr;
    }
    if (s->pool && r->ws_bytes && !keep_ws) s->pool->release(r->ws_off, r->ws_bytes);
    if (s->pool && r->ws_bytes && keep_ws)
        s->pending.push_back(psvt_server::Pending{r->lane, s->lanes[r->lane].tick - 1, r->ws_off, r->ws_bytes});
    r->ws_bytes = 0;
    r->plan.clear();
    r->plan.shrink_to_fit();
    if (state == RQ_DONE) {
        s->completed++;
        s->latency_ms.push_back(1e3 * (r->t_done - r->t_submit));
        s->queue_ms.push_back(1e3 * (r->t_admit - r->t_submit));
        s->last_done = r->t_done;
    } else {
        s->failed++;
    }
}

void worker_main(psvt_server *s) {
    if (!s->fake) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        const double t_now = now_s();
        // workspaces of failed requests whose lane has passed their stages
        for (size_t i = 0; i < s->pending.size();) {
            const psvt_server::Pending &p = s->pending[i];
            if (tick_passed(s, p.lane, p.tick)) {
                s->pool->release(p.off, p.bytes);
                s->pending[i] = s->pending.back();
                s->pending.pop_back();
            } else {
                ++i;
            }
        }
        // queued requests past their deadline fail without running
        if (s->timeout_s > 0.0) {
            bool any = false;
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                Request *r = *it;
                if (t_now - r->t_submit > s->timeout_s) {
                    r->ws_bytes = 0;  // never admitted: nothing in the pool
                    finish(s, r, RQ_FAILED);
                    s->timed_out++;
                    it = s->queue.erase(it);
                    any = true;
                } else {
                    ++it;
                }
            }
            if (any) s->cv_done.notify_all();
        }
        // admission: arrival order, one slot and pool room per request
        while (!s->queue.empty() && (int)s->active.size() < s->max_slots) {
            Request *r = s->queue.front();
            size_t off = 0;
            if (!s->pool->alloc(r->ws_bytes, &off)) break;  // wait for memory (no overtaking)
            r->ws_off = off;
            r->plan.clear();
            int rc = plan_request(r->op, r->item, s->fake ? (void *)(uintptr_t)(4096 + off) : s->pool_dev + off,
                                  &s->cfg, r->plan, &r->ws_bytes, !s->fake, r->cut);
            if (s->fake && s->plans++ == s->fault_plan) rc = set_error(PSVT_EINVAL, "injected planning failure");
            r->cursor = 0;
            r->curP = r->cut[0];
            r->curS = r->cut[1];
            s->queue.pop_front();
            r->t_admit = now_s();
            if (rc != PSVT_OK) {
                finish(s, r, RQ_FAILED);
                s->cv_done.notify_all();
                continue;
            }
            r->state = RQ_RUNNING;
            r->lane = lane_of(r->item, psvt_server::kLanes);
            if (s->cohort)  // a lane's running cohort is not joined half-way
                for (Request *o : s->active)
                    if (o->lane == r->lane && !o->parked && o->cursor > 0 && !plan_done(o)) {
                        r->parked = true;
                        break;
                    }
            s->active.push_back(r);
        }
        // completions, and active requests past their deadline (only this
        // request fails; its workspace waits for its lane's in-flight ticks)
        bool any_done = false;
        for (size_t i = 0; i < s->active.size();) {
            Request *r = s->active[i];
            bool done = false, late = false;
            if (r->finish_tick >= 0) done = s->fake ? !s->stall : tick_passed(s, r->lane, r->finish_tick);
            if (!done && s->timeout_s > 0.0 && t_now - r->t_submit > s->timeout_s) late = true;
            if (done || late) {
                if (done) {
                    finish(s, r, RQ_DONE);
                } else {
                    finish(s, r, RQ_FAILED, r->cursor + r->curP + r->curS > 0);
                    s->timed_out++;
                }
                s->active[i] = s->active.back();
                s->active.pop_back();
                any_done = true;
            } else {
                ++i;
            }
        }
        if (any_done) {
            s->cv_done.notify_all();
            continue;  // admit into the freed room first
        }
        // one tick per lane that has runnable requests and a free segment
        bool any_runnable = false, launched = false;
        for (int li = 0; li < psvt_server::kLanes; ++li) {
            psvt_server::Lane &ln = s->lanes[li];
            std::vector<Request *> runnable;
            for (Request *r : s->active)
                if (r->lane == li && !r->parked && !plan_done(r)) runnable.push_back(r);
            if (runnable.empty()) {  // the lane's cohort is through: the parked requests start together
                for (Request *r : s->active)
                    if (r->lane == li && r->parked) {
                        r->parked = false;
                        runnable.push_back(r);
                    }
            }
            if (runnable.empty()) continue;
            any_runnable = true;
            // one tick's descriptors must fit its segment: a round takes at
            // most two stages per request (descriptor + prefix entry each,
            // GemmArgs the largest descriptor) plus two 256-byte alignments
            // per group, and a round has at most 80 group keys (products:
            // 4 operand types x sym x two-operand x 4 tiles, norms, 4 tile
            // kinds); requests beyond that wait for the lane's next tick
            // (taken in rotation, so none waits for ever)
            static_assert(sizeof(GemmArgs) >= sizeof(NormOp) && sizeof(GemmArgs) >= sizeof(TileOp),
                          "GemmArgs is the largest descriptor");
            const size_t per_req = 2 * (sizeof(GemmArgs) + sizeof(int)) * (size_t)s->rounds;
            const size_t fixed = 2 * 256 * 80 * (size_t)s->rounds;
            const size_t cap = (psvt_server::kSegBytes - fixed) / per_req;
            if (runnable.size() > cap) {
                std::vector<Request *> win;
                for (size_t k = 0; k < cap; ++k) win.push_back(runnable[(ln.rr + k) % runnable.size()]);
                ln.rr = (ln.rr + cap) % runnable.size();
                runnable.swap(win);
            }
            // reuse the lane's oldest segment only once its tick has finished
            const int seg = (int)(ln.tick % s->nseg);
            if (!s->fake && ln.seg_tick[seg] >= 0 && hipEventQuery(ln.seg_event[seg]) != hipSuccess) continue;
            // order each newcomer after its submitter's stream; a request
            // whose wait cannot be enqueued fails alone (nothing of it ran)
            if (!s->fake) {
                std::vector<Request *> ok;
                for (Request *r : runnable) {
                    if (r->ready && !r->waited) {
                        if (hipStreamWaitEvent(ln.stream, r->ready, 0) != hipSuccess) {
                            (void)hipGetLastError();
                            finish(s, r, RQ_FAILED);
                            s->active.erase(std::find(s->active.begin(), s->active.end(), r));
                            s->cv_done.notify_all();
                            continue;
                        }
                        r->waited = true;
                    }
                    ok.push_back(r);
                }
                runnable.swap(ok);
                if (runnable.empty()) continue;
            }
            size_t seg_used = 0;
            int rc = PSVT_OK;
            std::vector<Group> gl;
            for (int round = 0; round < s->rounds && rc == PSVT_OK; ++round) {
                std::vector<Request *> rr;
                for (Request *r : runnable)
                    if (!plan_done(r)) rr.push_back(r);
                if (rr.empty()) break;
                rc = build_round(s, ln, rr, seg, seg_used, gl);
            }
            if (rc == PSVT_OK && s->fake && s->ticks == s->fault_tick)
                rc = set_error(PSVT_EHIP, "injected launch failure");
            if (rc == PSVT_OK) rc = launch_tick(s, ln, seg, seg_used, gl);
            if (!s->fake) {
                (void)hipEventRecord(ln.seg_event[seg], ln.stream);
                ln.seg_tick[seg] = ln.tick;
            }
            for (Request *r : runnable)
                if (plan_done(r) && r->finish_tick < 0) r->finish_tick = ln.tick;
            s->ticks++;
            ++ln.tick;
            launched = true;
            if (rc != PSVT_OK) {
                // this tick's launches are shared by its requests: they fail
                // (other lanes, and this lane's later requests, go on); the
                // lane's earlier ticks may still use their workspaces, which
                // return to the pool once those ticks have passed
                s->error = rc;
                for (Request *r : runnable) {
                    finish(s, r, RQ_FAILED, true);
                    s->active.erase(std::find(s->active.begin(), s->active.end(), r));
                }
                s->cv_done.notify_all();
            }
        }
        if (!any_runnable) {
            if (s->stop && s->queue.empty() && s->active.empty()) {
                if (!s->fake)
                    for (auto &ln : s->lanes) (void)hipStreamSynchronize(ln.stream);
                for (const psvt_server::Pending &p : s->pending) s->pool->release(p.off, p.bytes);
                s->pending.clear();
                break;
            }
            // wait for arrivals or for in-flight ticks to finish
            s->cv_work.wait_for(lk, std::chrono::microseconds(s->active.empty() ? 2000 : 50));
        } else if (!launched) {
            // every lane with work still has all its segments in flight
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double k = (v.size() - 1) * q;
    const size_t lo = (size_t)k, hi = std::min(v.size() - 1, lo + 1);
    return v[lo] + (v[hi] - v[lo]) * (k - lo);
}

}  // namespace

extern "C" {

int psvt_server_create(size_t budget_bytes, int32_t max_slots, const psvt_config *cfg, uint32_t flags,
                       psvt_server **out) {
    if (!out) return set_error(PSVT_EINVAL, "out is NULL");
    *out = nullptr;
    if (budget_bytes < 4096 || max_slots < 1 || max_slots > 4096)
        return set_error(PSVT_EINVAL, "bad budget or slot count");
    if (flags & ~(uint32_t)(PSVT_SERVER_FAKE | PSVT_SERVER_COHORT | PSVT_SERVER_EAGER))
        return set_error(PSVT_EINVAL, "unknown server flags");
    if ((flags & PSVT_SERVER_COHORT) && (flags & PSVT_SERVER_EAGER))
        return set_error(PSVT_EINVAL, "PSVT_SERVER_COHORT and PSVT_SERVER_EAGER exclude each other");
    if (cfg && (cfg->flags & PSVT_FLAG_STATUS))
        return set_error(PSVT_EINVAL, "PSVT_FLAG_STATUS names one status word per call, not per server");
    psvt_server *s = new psvt_server();
    s->fake = (flags & PSVT_SERVER_FAKE) != 0;
    s->cohort = (flags & PSVT_SERVER_EAGER) == 0;
    s->budget = budget_bytes;
    s->max_slots = max_slots;
    if (cfg) {
        s->cfg = *cfg;
        const int iters = cfg->iters ? cfg->iters : 20;
        if (cfg->coeffs) {
            s->coeffs.assign(cfg->coeffs, cfg->coeffs + 3 * iters);
            s->cfg.coeffs = s->coeffs.data();
        }
    }
    // descriptor rings: depth + 1 segments of 1 MiB per lane
    s->nseg = s->depth + 1;
    for (auto &ln : s->lanes) ln.seg_tick.assign(s->nseg, -1);
    s->pool = new Pool(budget_bytes);
    const size_t ring_bytes = psvt_server::kSegBytes * s->nseg * psvt_server::kLanes;
    if (!s->fake) {
        hipError_t e = hipGetDevice(&s->device);
        if (e == hipSuccess) e = hipMalloc((void **)&s->pool_dev, budget_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s->ring_host, ring_bytes, 0);
        if (e == hipSuccess) e = hipMalloc((void **)&s->ring_dev, ring_bytes);
        for (int li = 0; li < psvt_server::kLanes && e == hipSuccess; ++li) {
            psvt_server::Lane &ln = s->lanes[li];
            e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
            for (int i = 0; i < s->nseg && e == hipSuccess; ++i) {
                hipEvent_t ev;
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e == hipSuccess) ln.seg_event.push_back(ev);
            }
        }
        if (e != hipSuccess) {
            psvt_server_destroy(s);
            return set_error(PSVT_EHIP, hipGetErrorString(e));
        }
    } else {
        s->ring_host = (char *)malloc(ring_bytes);
        s->ring_dev = s->ring_host;
    }
    for (int li = 0; li < psvt_server::kLanes; ++li) {
        const size_t off = psvt_server::kSegBytes * s->nseg * li;
        s->lanes[li].ring_host = s->ring_host ? s->ring_host + off : nullptr;
        s->lanes[li].ring_dev = s->ring_dev ? s->ring_dev + off : nullptr;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return PSVT_OK;
}

int psvt_server_submit(psvt_server *s, int op, const psvt_batch_item *item, void *stream, uint64_t *ticket) {
    if (!s || !item || !ticket) return set_error(PSVT_EINVAL, "NULL argument");
    if (op != PSVT_OP_SVT && op != PSVT_OP_RANK_R) return set_error(PSVT_EINVAL, "op must be svt or rank_r");
    const psvt_batch_item &it = *item;
    if (it.m < 1 || it.n < 1 || !it.A || !it.Y || it.lda < it.n || it.ldy < it.n || !(it.tau >= 0.0) ||
        it.tau > 1e300)
        return set_error(PSVT_EINVAL, "bad request");
    Request *r = new Request();
    r->op = op;
    r->item = it;
    std::vector<Stage> none;
    size_t cut[3];
    int rc = plan_request(op, it, nullptr, &s->cfg, none, &r->ws_bytes, false, cut);
    if (rc != PSVT_OK) {
        delete r;
        return rc;
    }
    if (align256(r->ws_bytes) > s->budget) {
        delete r;
        return set_error(PSVT_EWORKSPACE, "request workspace exceeds the server's memory budget");
    }
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return set_error(PSVT_EINVAL, "server is shutting down");
        }
        if (!s->fake) {
            hipEvent_t ev = nullptr;
            hipError_t e = hipSuccess;
            if (!s->free_events.empty()) {
                ev = s->free_events.back();
                s->free_events.pop_back();
            } else {
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            }
            if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)stream);
            if (e != hipSuccess) {
                if (ev) s->free_events.push_back(ev);
                delete r;
                return set_error(PSVT_EHIP, hipGetErrorString(e));
            }
            r->ready = ev;
        }
        r->ticket = s->next_ticket++;
        s->all[r->ticket] = r;
        s->queue.push_back(r);
        s->submitted++;
        if (s->first_submit < 0) s->first_submit = r->t_submit;
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return PSVT_OK;
}

int psvt_server_poll(psvt_server *s, uint64_t ticket, int32_t *state) {
    if (!s || !state) return set_error(PSVT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(PSVT_EINVAL, "unknown ticket");
    *state = it->second->state;
    return PSVT_OK;
}

int psvt_server_wait(psvt_server *s, uint64_t ticket, double timeout_s, int32_t *state) {
    if (!s) return set_error(PSVT_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return set_error(PSVT_EINVAL, "unknown ticket");
    Request *r = it->second;
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (r->state == RQ_QUEUED || r->state == RQ_RUNNING)
        if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout) break;
    if (state) *state = r->state;
    return PSVT_OK;
}

int psvt_server_drain(psvt_server *s, double timeout_s) {
    if (!s) return set_error(PSVT_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (!s->queue.empty() || !s->active.empty())
        if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout)
            return set_error(PSVT_EINVAL, "drain timed out");
    if (s->error != PSVT_OK)  // the worker's message is on its own thread
        return set_error(s->error, "a launch failed in the server: the requests of that tick failed");
    return PSVT_OK;
}

int psvt_server_stats(psvt_server *s, psvt_server_counters *st) {
    if (!s || !st) return set_error(PSVT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof *st);
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->timed_out = s->timed_out;
    st->queued = (int64_t)s->queue.size();
    st->active = (int64_t)s->active.size();
    st->ticks = s->ticks;
    st->launches = s->launches;
    st->p50_ms = percentile(s->latency_ms, 0.5);
    st->p99_ms = percentile(s->latency_ms, 0.99);
    st->max_ms = s->latency_ms.empty() ? 0.0 : *std::max_element(s->latency_ms.begin(), s->latency_ms.end());
    st->queue_p99_ms = percentile(s->queue_ms, 0.99);
    const double span = s->last_done - s->first_submit;
    st->matrices_per_s = (s->completed > 0 && span > 0) ? s->completed / span : 0.0;
    st->budget_bytes = s->budget;
    st->peak_bytes = s->pool->peak();
    return PSVT_OK;
}

int psvt_server_set_timeout(psvt_server *s, double seconds) {
    if (!s) return set_error(PSVT_EINVAL, "NULL server");
    if (!(seconds >= 0.0) || seconds > 1e9) return set_error(PSVT_EINVAL, "timeout outside [0, 1e9] seconds");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->timeout_s = seconds;
    }
    s->cv_work.notify_all();
    return PSVT_OK;
}

int psvt_server_inject_fault(psvt_server *s, int kind, int64_t n) {
    if (!s) return set_error(PSVT_EINVAL, "NULL server");
    if (!s->fake) return set_error(PSVT_EINVAL, "fault injection is for PSVT_SERVER_FAKE servers");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        switch (kind) {
            case PSVT_FAULT_TICK: s->fault_tick = n; break;
            case PSVT_FAULT_PLAN: s->fault_plan = n; break;
            case PSVT_FAULT_STALL: s->stall = n != 0; break;
            default: return set_error(PSVT_EINVAL, "unknown fault kind");
        }
    }
    s->cv_work.notify_all();
    return PSVT_OK;
}

int psvt_server_destroy(psvt_server *s) {
    if (!s) return PSVT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (!s->fake) {
        for (auto &ln : s->lanes) {
            if (ln.stream) (void)hipStreamSynchronize(ln.stream);
            for (hipEvent_t e : ln.seg_event) (void)hipEventDestroy(e);
            if (ln.stream) (void)hipStreamDestroy(ln.stream);
        }
        if (s->ring_dev) (void)hipFree(s->ring_dev);
        if (s->ring_host) (void)hipHostFree(s->ring_host);
        if (s->pool_dev) (void)hipFree(s->pool_dev);
    } else {
        free(s->ring_host);
    }
    for (auto &kv : s->all) {
        if (kv.second->ready) s->free_events.push_back(kv.second->ready);
        delete kv.second;
    }
    if (!s->fake)
        for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    delete s->pool;
    delete s;
    return PSVT_OK;
}

}  // extern "C"
