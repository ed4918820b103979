// Column-tile copy: the HBM access pattern of the fused z passes with no
// transform.  A field of packed spectra is C columns of nz complex values,
// z-major (element (z, c) at z C + c).  A block copies a tile of tb adjacent
// columns: each of its tb * nz / E threads owns column b = tid % tb and the
// elements z = t + m L (t = tid / tb, L = nz / E, m < E), loads all of them,
// optionally passes them through one LDS exchange (write, barrier, read in
// another thread order, and back), and stores them.  Every row of a tile is
// tb * 8 contiguous bytes, and consecutive rows lie C * 8 bytes apart, as in
// the z passes.  The timing of this copy is the ceiling of a z pass that
// moves the same bytes in the same tiles.  Each timed launch follows a read of
// 1 GiB of other memory, so that it starts with cold caches.
//
// Usage: zcol_copy  (prints one Markdown table row per configuration)
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                          \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                              \
        }                                                                              \
    } while (0)

template <int E, bool XCHG>
__global__ void __launch_bounds__(512) zcol_copy(const float2 *__restrict__ in, float2 *__restrict__ out,
                                                 long C, int nz, int tb) {
    extern __shared__ float2 sh[];
    const int L = nz / E;
    const int b = threadIdx.x % tb, t = threadIdx.x / tb;
    const long col = (long)blockIdx.x * tb + b;
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = in[(long)(t + m * L) * C + col];
    if (XCHG) {
#pragma unroll
        for (int m = 0; m < E; ++m) sh[(t + m * L) * tb + b] = v[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = sh[(t * E + m) * tb + b];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) sh[(t * E + m) * tb + b] = v[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = sh[(t + m * L) * tb + b];
    }
#pragma unroll
    for (int m = 0; m < E; ++m) out[(long)(t + m * L) * C + col] = v[m];
}

// Reads a buffer larger than the caches (L2 and the 256 MB last-level cache)
// before each timed copy, so that the copy's loads come from HBM.  The sum is
// written only if it is an impossible value, which keeps the loads alive.
__global__ void __launch_bounds__(256) evict(const float4 *__restrict__ p, size_t n, float *sink) {
    float s = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float4 v = p[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == -1.0f) *sink = s;
}

static const float4 *g_evict = nullptr;
static size_t g_evict_n = 0;
static float *g_sink = nullptr;

static void evict_caches() {
    hipLaunchKernelGGL(evict, dim3(4096), dim3(256), 0, 0, g_evict, g_evict_n, g_sink);
    CK(hipGetLastError());
}

static float time_ms(hipEvent_t a, hipEvent_t z) {
    float ms = 0.0f;
    CK(hipEventElapsedTime(&ms, a, z));
    return ms;
}

template <int E, bool XCHG>
static void run(const float2 *in, float2 *out, long C, int nz, int tb, const char *grid) {
    const int threads = tb * (nz / E);
    // every index stays inside the C * nz elements of a field: col < C because
    // C is a multiple of tb, and t + m L < nz, t E + m < nz because t < L
    if (threads > 512 || threads < 64 || C % tb != 0 || nz % E != 0) return;
    const size_t lds = XCHG ? (size_t)tb * nz * 8 : 0;
    if (lds > 160 * 1024) return;
    const long blocks = C / tb;
    hipEvent_t a, z;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&z));
    hipLaunchKernelGGL((zcol_copy<E, XCHG>), dim3(blocks), dim3(threads), lds, 0, in, out, C, nz, tb);
    CK(hipGetLastError());
    CK(hipDeviceSynchronize());
    const double bytes = 2.0 * (double)C * nz * 8;
    const int reps = 5;
    float ms = 0.0f;
    for (int r = 0; r < reps; ++r) {
        evict_caches();
        CK(hipEventRecord(a));
        hipLaunchKernelGGL((zcol_copy<E, XCHG>), dim3(blocks), dim3(threads), lds, 0, in, out, C, nz, tb);
        CK(hipGetLastError());
        CK(hipEventRecord(z));
        CK(hipEventSynchronize(z));
        ms += time_ms(a, z) / reps;
    }
    std::printf("| %s | %d | %d | %d | %d | %d | %s | %.3f | %.2f |\n", grid, tb, tb * 8, E, threads,
                (int)(lds / 1024), XCHG ? "yes" : "no", ms, bytes / ms / 1e9);
    std::fflush(stdout);
    CK(hipEventDestroy(a));
    CK(hipEventDestroy(z));
}

int main() {
    const size_t n = 512ul * 1024 * 1024;   // complex values of the largest field (4 GiB)
    float2 *in = nullptr, *out = nullptr;
    CK(hipMalloc(&in, n * 8));
    CK(hipMalloc(&out, n * 8));
    CK(hipMemset(in, 0, n * 8));
    g_evict_n = (1ul << 30) / sizeof(float4);   // 1 GiB
    float4 *ev = nullptr;
    CK(hipMalloc(&ev, g_evict_n * sizeof(float4)));
    CK(hipMemset(ev, 0, g_evict_n * sizeof(float4)));
    CK(hipMalloc(&g_sink, sizeof(float)));
    g_evict = ev;
    std::printf("| grid (columns x nz) | tile columns | bytes per row | E | threads | LDS KiB | exchange | ms | TB/s |\n");
    std::printf("|---|---|---|---|---|---|---|---|---|\n");
    struct Shape { long C; int nz; const char *name; };
    const Shape shapes[] = {{512l * 1024, 1024, "512x1024 x 1024 (1024^3)"},
                            {128l * 256, 256, "128x256 x 256 (256^3)"}};
    for (const Shape &s : shapes) {
        for (int tb : {4, 8, 16}) {
            run<16, false>(in, out, s.C, s.nz, tb, s.name);
            run<16, true>(in, out, s.C, s.nz, tb, s.name);
            run<32, false>(in, out, s.C, s.nz, tb, s.name);
            run<32, true>(in, out, s.C, s.nz, tb, s.name);
        }
    }
    hipEvent_t a, z;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&z));
    CK(hipMemcpyAsync(out, in, n * 8, hipMemcpyDeviceToDevice, 0));
    CK(hipEventRecord(a));
    for (int r = 0; r < 5; ++r) CK(hipMemcpyAsync(out, in, n * 8, hipMemcpyDeviceToDevice, 0));
    CK(hipEventRecord(z));
    CK(hipEventSynchronize(z));
    const float ms = time_ms(a, z) / 5;
    std::printf("\ncontiguous device-to-device copy of 4 GiB: %.3f ms, %.2f TB/s\n", ms, 2.0 * n * 8 / ms / 1e9);
    CK(hipFree(in));
    CK(hipFree(out));
    CK(hipFree(ev));
    CK(hipFree(g_sink));
    return 0;
}
