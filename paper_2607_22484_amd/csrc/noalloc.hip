// psvt_svt_noalloc: soft-thresholding with no device allocation at all, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The workspace is `scratch`, a file-scope device array of
// PSVT_NOALLOC_SCRATCH_BYTES per device, held until the process ends.  Host
// code never passes the array's name to a kernel (in host code it is a
// host-side stand-in, not a device address): once per device, with that
// device current, the library asks the runtime for the array's address
// (hipGetSymbolAddress) and keeps it; every launch then takes that address.
// The plan is psvt_svt's (same kernels, same results), with every launch on
// the caller's stream: no side stream, no event, nothing created.  No buffer
// of the plan needs to start at zero (every one is written before it is
// read), so the array is never cleared; calls that overlap on one device
// share it and race.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/psvt.h"

namespace psvt {
int svt_on_workspace(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy,
                     void *ws, size_t ws_bytes, const psvt_config *cfg, void *stream);
int svt_workspace_unforked(int64_t m, int64_t n, const psvt_config *cfg, size_t *bytes);
int set_error(int code, const char *msg);
}  // namespace psvt

namespace {

static __device__ __align__(256) unsigned char scratch[PSVT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// The device address of this device's `scratch`, looked up once per device
// (with that device current); NULL with the message set on failure.
void *scratch_address(int *rc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *rc = psvt::set_error(PSVT_EHIP, hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *rc = psvt::set_error(PSVT_EUNSUPPORTED, "device index out of range");
        return nullptr;
    }
    std::call_once(g_once[dev], [dev]() {
        void *p = nullptr;
        g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
    });
    if (g_err[dev] != hipSuccess || !g_ptr[dev]) {
        *rc = psvt::set_error(PSVT_EHIP, g_err[dev] != hipSuccess ? hipGetErrorString(g_err[dev])
                                                                   : "no address for the scratch array");
        return nullptr;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

int psvt_svt_noalloc(const float *A, int64_t m, int64_t n, int64_t lda, double tau, float *Y, int64_t ldy,
                     const psvt_config *cfg, void *stream) {
    size_t need = 0;
    int rc = psvt::svt_workspace_unforked(m < 0 ? 0 : m, n < 0 ? 0 : n, cfg, &need);
    if (rc) return rc;
    if (need > (size_t)PSVT_NOALLOC_SCRATCH_BYTES)
        return psvt::set_error(PSVT_EWORKSPACE,
                               "psvt_svt_noalloc: this size and schedule need more workspace than the "
                               "PSVT_NOALLOC_SCRATCH_BYTES static scratch (use psvt_svt with a caller workspace)");
    void *ws = nullptr;
    if (m > 0 && n > 0) {
        rc = PSVT_OK;
        if (!(ws = scratch_address(&rc))) return rc;
    }
    return psvt::svt_on_workspace(A, m, n, lda, tau, Y, ldy, ws, PSVT_NOALLOC_SCRATCH_BYTES, cfg, stream);
}

}  // extern "C"
