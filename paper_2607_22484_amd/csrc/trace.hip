// Launch tracing: see trace.h and psvt_trace_begin / psvt_trace_end.
#include "trace.h"

#include <string.h>

#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/psvt.h"

namespace psvt {
namespace {

struct Rec {
    const char *name;
    double flops, bytes;
    hipEvent_t start, stop;
};

struct State {
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;  // idle events, reused across sessions
    hipEvent_t get() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
};

thread_local State g_state;

}  // namespace

bool trace_on() { return g_state.on; }

const char *trace_name(const char *name) {
    static std::mutex mu;
    static std::unordered_set<std::string> *names = new std::unordered_set<std::string>();
    std::lock_guard<std::mutex> lock(mu);
    return names->insert(name).first->c_str();
}

TraceScope::TraceScope(hipStream_t st, const char *name, double flops, double bytes)
    : st_(st), name_(name), flops_(flops), bytes_(bytes) {
    if (!g_state.on) return;
    start_ = g_state.get();
    stop_ = g_state.get();
    if (start_) (void)hipEventRecord(start_, st_);
}

TraceScope::~TraceScope() {
    if (!start_ || !stop_) {
        if (start_) g_state.pool.push_back(start_);
        if (stop_) g_state.pool.push_back(stop_);
        return;
    }
    (void)hipEventRecord(stop_, st_);
    g_state.recs.push_back(Rec{name_, flops_, bytes_, start_, stop_});
}

}  // namespace psvt

using namespace psvt;

extern "C" {

int psvt_trace_begin(void) {
    for (auto &r : g_state.recs) {
        g_state.pool.push_back(r.start);
        g_state.pool.push_back(r.stop);
    }
    g_state.recs.clear();
    g_state.on = true;
    return PSVT_OK;
}

int psvt_trace_end(psvt_trace_stat *out, int max_entries, int *n_entries) {
    g_state.on = false;
    std::vector<psvt_trace_stat> agg;
    int rc = PSVT_OK;
    for (auto &r : g_state.recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.stop) != hipSuccess || hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            rc = PSVT_EHIP;
        size_t k = 0;
        while (k < agg.size() && strcmp(agg[k].name, r.name) != 0) ++k;
        if (k == agg.size()) {
            psvt_trace_stat z;
            memset(&z, 0, sizeof z);
            z.name = r.name;
            agg.push_back(z);
        }
        agg[k].launches += 1;
        agg[k].total_ms += ms;
        agg[k].flops += r.flops;
        agg[k].bytes += r.bytes;
        g_state.pool.push_back(r.start);
        g_state.pool.push_back(r.stop);
    }
    g_state.recs.clear();
    // most time first
    for (size_t i = 1; i < agg.size(); ++i)
        for (size_t j = i; j > 0 && agg[j].total_ms > agg[j - 1].total_ms; --j) std::swap(agg[j], agg[j - 1]);
    int n = 0;
    for (size_t i = 0; i < agg.size() && (out && n < max_entries); ++i) out[n++] = agg[i];
    if (n_entries) *n_entries = out ? n : (int)agg.size();
    return rc;
}

}  // extern "C"
