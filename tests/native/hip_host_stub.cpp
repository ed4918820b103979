// Host stand-in for the HIP runtime and the library's kernel launchers, for
// building the engine's host code on a machine without a GPU (under
// AddressSanitizer or ThreadSanitizer).  "Device memory" is host memory:
// copies are memcpy, the fill launchers write the values, every other
// launcher does nothing.  kw_stub_fail_launches makes every launcher and copy
// fail with hipErrorLaunchFailure (error propagation tests).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>

#include "kw_internal.h"

extern "C" {
std::atomic<int> kw_stub_fail_launches{0};
}

static hipError_t launch_status() {
    return kw_stub_fail_launches.load() ? hipErrorLaunchFailure : hipSuccess;
}

extern "C" {
hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) { *v = 160 * 1024; return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "stub error"; }
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t) {
    if (launch_status() != hipSuccess) return launch_status();
    std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k) {
    return hipMemcpyAsync(dst, src, n, k, nullptr);
}
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t) {
    std::memset(dst, v, n);
    return launch_status();
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = nullptr; return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, hipGraphNode_t *, char *, size_t) {
    return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = nullptr; return hipErrorNotSupported; }
hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.0f; return hipErrorNotSupported; }
}

namespace kw {

// the static scratch array stands in as host memory here
hipError_t static_scratch(void **out, size_t *bytes) {
    alignas(256) static unsigned char host_scratch[1 << 20];
    *out = host_scratch;
    *bytes = sizeof host_scratch;
    return launch_status();
}

hipError_t launch_fill(hipStream_t, float *p, size_t n, float v) {
    for (size_t i = 0; i < n; ++i) p[i] = v;
    return launch_status();
}
hipError_t launch_fill_int(hipStream_t, int *p, size_t n, int v) {
    for (size_t i = 0; i < n; ++i) p[i] = v;
    return launch_status();
}
hipError_t launch_ypass(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &,
                        float2 *const *, int, bool, const Counters *, const SourceDev *,
                        const SensorDev *, float2 *const *) { return launch_status(); }
hipError_t launch_zfused(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &, int,
                         float2 *const *, float2 *const *, float, float, float2 *const *) {
    return launch_status();
}
hipError_t launch_xvel(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &,
                       const Medium &, float2 *const *, float *const *, const SourceDev &,
                       const SensorDev &, const Counters &) { return launch_status(); }
hipError_t launch_xden(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &,
                       const Medium &, const SourceDev &, const SensorDev &, const Counters &,
                       float2 *const *, float *const *, float *, float2 *const *, bool,
                       float *const *) {
    return launch_status();
}
hipError_t launch_xeos(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &,
                       const Medium &, const SourceDev &, const SensorDev &, const Counters &,
                       float2 *const *, const float *, float2 *, bool) { return launch_status(); }
hipError_t launch_xfwd(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &,
                       const float *, float2 *) { return launch_status(); }
hipError_t launch_xinv(hipStream_t, const GridDev &, const LaunchCfg &, const Tables &,
                       const float2 *, float *, float) { return launch_status(); }
hipError_t launch_adj_weights(hipStream_t, const GridDev &, const Medium &, float *, float) {
    return launch_status();
}
hipError_t launch_adj_src(hipStream_t, const AdjDev &, const SourceDev &, int) {
    return launch_status();
}
hipError_t launch_adj_src_sum(hipStream_t, const AdjDev &, int) { return launch_status(); }
hipError_t launch_adjx(hipStream_t, int, const GridDev &, const LaunchCfg &, const Tables &,
                       const Medium &, const SourceDev &, const AdjDev &, const float2 *, bool,
                       float2 *const *, float2 *const *) {
    return launch_status();
}
int adj_objective_blocks(const GridDev &g) {
    return (int)std::min<size_t>(((size_t)g.nx * g.rows + 255) / 256, 65535u * 8u);
}
hipError_t launch_adj_objective(hipStream_t, const GridDev &, const float *, const float *,
                                double *, double *) { return launch_status(); }
hipError_t launch_scale(hipStream_t, const float *, float *, size_t, float) { return launch_status(); }
hipError_t launch_finalize(hipStream_t, const float *, float *, size_t, float, int, Coef, Coef,
                           const int *) { return launch_status(); }

}  // namespace kw
