// Small utility kernels: fills and the gather-time finalisation of sensors.
#include "kernels_impl.h"

namespace kw {

__global__ void kw_fill(float *p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void kw_scale(const float *src, float *dst, size_t n, float scale) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i] * scale;
}

__global__ void kw_fill_int(int *p, size_t n, int v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
// mode 0: sqrt(sum2 * inv_count) (p_rms); mode 1: sum2 * inv_count / (rho0 c0) (intensity)
__global__ void kw_finalize(const float *sum2, float *dst, size_t n, float inv_count, int mode,
                            Coef rho0, Coef c0sq, const int *index) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float m = sum2[i] * inv_count;
        if (mode == 0) {
            dst[i] = sqrtf(m);
        } else {
            const size_t g = index ? (size_t)index[i] : i;
            dst[i] = m / (coef_at(rho0, g) * sqrtf(coef_at(c0sq, g)));
        }
    }
}

static inline dim3 flat_grid(size_t n) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    return dim3((unsigned)blocks);
}

hipError_t launch_fill(hipStream_t s, float *p, size_t n, float v) {
    hipLaunchKernelGGL(kw_fill, flat_grid(n), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_scale(hipStream_t s, const float *src, float *dst, size_t n, float scale) {
    hipLaunchKernelGGL(kw_scale, flat_grid(n), dim3(256), 0, s, src, dst, n, scale);
    return hipGetLastError();
}
hipError_t launch_fill_int(hipStream_t s, int *p, size_t n, int v) {
    hipLaunchKernelGGL(kw_fill_int, flat_grid(n), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_finalize(hipStream_t s, const float *sum2, float *dst, size_t n, float inv_count,
                           int mode, Coef rho0, Coef c0sq, const int *index) {
    hipLaunchKernelGGL(kw_finalize, flat_grid(n), dim3(256), 0, s, sum2, dst, n, inv_count, mode,
                       rho0, c0sq, index);
    return hipGetLastError();
}

}  // namespace kw
