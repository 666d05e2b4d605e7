// Per-launch event tracing (enabled by psvt_trace_begin on the calling
// thread).  Each traced launch is bracketed by two HIP events recorded on the
// launch's own stream, so the elapsed time is that kernel's device time.
#pragma once
#include <hip/hip_runtime.h>

namespace psvt {

bool trace_on();

// Interned copy of `name` that lives until the process ends.
const char *trace_name(const char *name);

class TraceScope {
  public:
    TraceScope(hipStream_t st, const char *name, double flops, double bytes);
    ~TraceScope();
    TraceScope(const TraceScope &) = delete;
    TraceScope &operator=(const TraceScope &) = delete;

  private:
    hipStream_t st_;
    const char *name_;
    double flops_, bytes_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
};

}  // namespace psvt
