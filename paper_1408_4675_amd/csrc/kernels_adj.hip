// Point-wise pieces of the reverse-mode (discrete adjoint) step.  The
// spectral pieces reuse the forward passes (x r2c / c2r, y pass, fused z pass
// with the transposed operators); the host sequence is in engine.cpp.
//
// The step being reversed is step n of Eqs. (4a)-(4d), (6), (8):
//   g_xi  = IFT(D+_xi kappa FT p),         u_xi' = q+ (q+ u_xi - dt/rho0+ g_xi)
//   d_xi  = IFT(D-_xi kappa FT u_xi'),      rho_xi' = q (q rho_xi - dt rho0 d_xi) / den_xi + src
//   den_xi = 1 + 2 dt d_xi (nonlinear),     rho = sum rho_xi'
//   p' = c0^2 rho + nl rho^2 + ta a + tb b, a = IFT(k^(y-2) FT(rho0 sum d)), b = IFT(k^(y-1) FT rho)
// with nl = c0^2 B/A / (2 rho0), ta = c0^2 tau, tb = -c0^2 eta.  Given the
// adjoints pb, ub, rb of (p', u', rho') the kernels below form, in order:
//   eos:  pbar = pb + w p' (recorded steps),  rbt = (c0^2 + 2 nl rho) pbar,
//         T0 = ta pbar, T1 = tb pbar           (then T0 <- A T0, T1 <- B T1 spectrally)
//   src:  at source points, R_xi = rb_xi + rbt + T1, the point's share coef sum_xi R_xi
//         of dJ/ds_e(n) and the correction 2 dt R_xi src / den_xi of the
//         divergence adjoint; the shares of each element are then summed in a
//         fixed order (no floating-point atomics: the gradient is repeatable
//         bit for bit)
//   den:  R_xi = rb_xi + rbt + T1,  rb_xi <- R_xi q^2 / den_xi,
//         d_xi <- -R_xi (q dt rho0 + 2 dt rho_xi') / den_xi + rho0 T0
//   (spectral: T_xi = transpose-divergence of d_xi)
//   vel:  u = ub_xi + T_xi,  T_xi <- -q+ dt/rho0+ u,  ub_xi <- q+^2 u
//   (spectral: T_xi = transpose-gradient of T_xi)
//   sum:  pb = T0 + T1 + T2
#include "kernels_impl.h"

namespace kw {

namespace {

constexpr int kThreads = 256;

inline dim3 grid_for(size_t n) {
    const size_t b = (n + kThreads - 1) / kThreads;
    return dim3((unsigned)std::min<size_t>(b, 65535u * 8u));
}

__device__ __forceinline__ size_t npoints(const GridDev &g) { return (size_t)g.nx * g.rows; }

}  // namespace

__global__ void __launch_bounds__(kThreads) kw_adj_weights(GridDev g, Medium m, float *w, float scale) {
    const size_t N = npoints(g);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        const float rc = coef_at(m.rho0, i) * sqrtf(coef_at(m.c0sq, i));
        w[i] = scale * w[i] / rc;
    }
}

__global__ void __launch_bounds__(kThreads) kw_adj_eos(GridDev g, Medium m, AdjDev a, int loss) {
    const size_t N = npoints(g);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        float pbar = a.pb[i];
        if (loss) pbar += a.w[i] * a.pf[i];
        float c = coef_at(m.c0sq, i);
        if (m.nonlinear) c += 2.0f * coef_at(m.nl, i) * (a.rho[0][i] + a.rho[1][i] + a.rho[2][i]);
        a.rbt[i] = c * pbar;
        if (m.absorbing) {
            a.T[0][i] = coef_at(m.ta, i) * pbar;
            a.T[1][i] = coef_at(m.tb, i) * pbar;
        }
    }
}

__global__ void __launch_bounds__(kThreads) kw_adj_src(GridDev g, Medium m, AdjDev a,
                                                        SourceDev src, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_src) return;
    const size_t f = (size_t)a.src_flat[k];
    const int e = a.src_elem[k];
    const float coef = a.src_coef[k];
    const float add = coef * drive_at(src, e, n);
    const float base = a.rbt[f] + (m.absorbing ? a.T[1][f] : 0.0f);
    float rsum = 0.0f;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        const float R = pick3v(a.rb[0], a.rb[1], a.rb[2], x)[f] + base;
        rsum += R;
        float c = 0.0f;
        if (m.nonlinear) {
            const float den = 1.0f + 2.0f * g.dt * pick3v(a.dfw[0], a.dfw[1], a.dfw[2], x)[f];
            c = R * 2.0f * g.dt * add / den;
        }
        a.corr[(size_t)x * a.n_src + k] = c;
    }
    a.share[k] = (double)coef * (double)rsum;
}

// Sum of block-sized slices in a fixed order: each thread adds the values it
// strides over, then a fixed tree over the block.  Called by every thread.
__device__ __forceinline__ double block_sum(double v, double *part) {
    part[threadIdx.x] = v;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    const double r = part[0];
    __syncthreads();
    return r;
}

// dJ/ds_e(n) = sum of the shares of element e's points (one block per element,
// points in the order of the element's list)
__global__ void __launch_bounds__(kThreads) kw_adj_src_sum(AdjDev a, int n) {
    __shared__ double part[kThreads];
    const int e = blockIdx.x;
    double acc = 0.0;
    for (int j = a.elem_ptr[e] + (int)threadIdx.x; j < a.elem_ptr[e + 1]; j += kThreads)
        acc += a.share[a.elem_pts[j]];
    const double total = block_sum(acc, part);
    if (threadIdx.x == 0) a.dJds[(size_t)n * a.n_elem + e] = total;
}

__global__ void __launch_bounds__(kThreads) kw_adj_den(GridDev g, Tables t, Medium m, AdjDev a) {
    const size_t N = npoints(g);
    const float dt = g.dt;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        const int ix = (int)(i % g.nx);
        const size_t row = i / g.nx;
        const int iy = (int)(row % g.ny), iz = (int)(row / g.ny);
        const float rbt = a.rbt[i] + (m.absorbing ? a.T[1][i] : 0.0f);
        const float rho0 = coef_at(m.rho0, i);
        const float dcom = m.absorbing ? rho0 * a.T[0][i] : 0.0f;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const float q = x == 0 ? t.pml_x[ix] : x == 1 ? t.pml_y[iy] : t.pml_z[iz];
            float *rb = pick3v(a.rb[0], a.rb[1], a.rb[2], x);
            float *d = pick3v(a.d[0], a.d[1], a.d[2], x);
            const float R = rb[i] + rbt;
            float den = 1.0f, dbar;
            if (m.nonlinear) {
                den = 1.0f + 2.0f * dt * pick3v(a.dfw[0], a.dfw[1], a.dfw[2], x)[i];
                const float rn = pick3v(a.rho[0], a.rho[1], a.rho[2], x)[i];
                dbar = -R * (q * dt * rho0 + 2.0f * dt * rn) / den;
            } else {
                dbar = -R * q * dt * rho0;
            }
            rb[i] = R * q * q / den;
            d[i] = dbar + dcom;
        }
    }
}

__global__ void __launch_bounds__(kThreads) kw_adj_src_fix(AdjDev a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_src) return;
    const size_t f = (size_t)a.src_flat[k];
#pragma unroll
    for (int x = 0; x < 3; ++x) pick3v(a.d[0], a.d[1], a.d[2], x)[f] += a.corr[(size_t)x * a.n_src + k];
}

__global__ void __launch_bounds__(kThreads) kw_adj_vel(GridDev g, Tables t, Medium m, AdjDev a) {
    const size_t N = npoints(g);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        const int ix = (int)(i % g.nx);
        const size_t row = i / g.nx;
        const int iy = (int)(row % g.ny), iz = (int)(row / g.ny);
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const float q = x == 0 ? t.pml_sx[ix] : x == 1 ? t.pml_sy[iy] : t.pml_sz[iz];
            const Coef dtr = x == 0 ? m.dtr[0] : x == 1 ? m.dtr[1] : m.dtr[2];
            float *ub = pick3v(a.ub[0], a.ub[1], a.ub[2], x);
            float *T = pick3v(a.T[0], a.T[1], a.T[2], x);
            const float u = ub[i] + T[i];
            T[i] = -q * coef_at(dtr, i) * u;
            ub[i] = q * q * u;
        }
    }
}

__global__ void __launch_bounds__(kThreads) kw_adj_sum(GridDev g, AdjDev a) {
    const size_t N = npoints(g);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x)
        a.pb[i] = a.T[0][i] + a.T[1][i] + a.T[2][i];
}

// J = 1/2 sum_i w'(i) sum2(i) with w' = 2 w / (rho0 c0 N_w): block sums in
// float64 into partials[blockIdx.x], then one block adds the partials in order
__global__ void __launch_bounds__(kThreads) kw_adj_objective(GridDev g, const float *w,
                                                              const float *sum2, double *partials) {
    __shared__ double part[kThreads];
    const size_t N = npoints(g);
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x)
        acc += 0.5 * (double)w[i] * (double)sum2[i];
    const double total = block_sum(acc, part);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) kw_adj_partials(const double *partials, int n,
                                                             double *out) {
    __shared__ double part[kThreads];
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += kThreads) acc += partials[j];
    const double total = block_sum(acc, part);
    if (threadIdx.x == 0) *out = total;
}

// launchers -----------------------------------------------------------------------

int adj_objective_blocks(const GridDev &g) { return (int)grid_for((size_t)g.nx * g.rows).x; }

hipError_t launch_adj_objective(hipStream_t s, const GridDev &g, const float *w,
                                const float *sum2, double *partials, double *out) {
    const size_t N = (size_t)g.nx * g.rows;
    const dim3 grid = grid_for(N);
    hipLaunchKernelGGL(kw_adj_objective, grid, dim3(kThreads), 0, s, g, w, sum2, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kw_adj_partials, dim3(1), dim3(kThreads), 0, s, partials, (int)grid.x, out);
    return hipGetLastError();
}


hipError_t launch_adj_weights(hipStream_t s, const GridDev &g, const Medium &m, float *w,
                              float scale) {
    const size_t N = (size_t)g.nx * g.rows;
    hipLaunchKernelGGL(kw_adj_weights, grid_for(N), dim3(kThreads), 0, s, g, m, w, scale);
    return hipGetLastError();
}

hipError_t launch_adj_eos(hipStream_t s, const GridDev &g, const Medium &m, const AdjDev &a,
                          bool loss) {
    const size_t N = (size_t)g.nx * g.rows;
    hipLaunchKernelGGL(kw_adj_eos, grid_for(N), dim3(kThreads), 0, s, g, m, a, loss ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_adj_src(hipStream_t s, const GridDev &g, const Medium &m, const AdjDev &a,
                          const SourceDev &src, int n) {
    if (a.n_src == 0) return hipSuccess;
    hipLaunchKernelGGL(kw_adj_src, dim3((a.n_src + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                       g, m, a, src, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kw_adj_src_sum, dim3(a.n_elem), dim3(kThreads), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_adj_den(hipStream_t s, const GridDev &g, const Tables &t, const Medium &m,
                          const AdjDev &a) {
    const size_t N = (size_t)g.nx * g.rows;
    hipLaunchKernelGGL(kw_adj_den, grid_for(N), dim3(kThreads), 0, s, g, t, m, a);
    return hipGetLastError();
}

hipError_t launch_adj_src_fix(hipStream_t s, const AdjDev &a, const Medium &m) {
    if (a.n_src == 0 || !m.nonlinear) return hipSuccess;
    hipLaunchKernelGGL(kw_adj_src_fix, dim3((a.n_src + kThreads - 1) / kThreads), dim3(kThreads),
                       0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_vel(hipStream_t s, const GridDev &g, const Tables &t, const Medium &m,
                          const AdjDev &a) {
    const size_t N = (size_t)g.nx * g.rows;
    hipLaunchKernelGGL(kw_adj_vel, grid_for(N), dim3(kThreads), 0, s, g, t, m, a);
    return hipGetLastError();
}

hipError_t launch_adj_sum(hipStream_t s, const GridDev &g, const AdjDev &a) {
    const size_t N = (size_t)g.nx * g.rows;
    hipLaunchKernelGGL(kw_adj_sum, grid_for(N), dim3(kThreads), 0, s, g, a);
    return hipGetLastError();
}

}  // namespace kw
