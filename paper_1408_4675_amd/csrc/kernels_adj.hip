// Reverse-mode (discrete adjoint) step: fused x-row passes, point-wise source
// pieces and the objective.  The spectral pieces between the x passes are the
// forward y passes and the fused z pass with the transposed operators; the
// host sequence is in engine.cpp.
//
// The step being reversed is step n of Eqs. (4a)-(4d), (6), (8):
//   g_xi  = IFT(D+_xi kappa FT p),         u_xi' = q+ (q+ u_xi - dt/rho0+ g_xi)
//   d_xi  = IFT(D-_xi kappa FT u_xi'),      rho_xi' = q (q rho_xi - dt rho0 d_xi) / den_xi + src
//   den_xi = 1 + 2 dt d_xi (nonlinear),     rho = sum rho_xi'
//   p' = c0^2 rho + nl rho^2 + ta a + tb b, a = IFT(k^(y-2) FT(rho0 sum d)), b = IFT(k^(y-1) FT rho)
// with nl = c0^2 B/A / (2 rho0), ta = c0^2 tau, tb = -c0^2 eta.  Given the
// adjoints pb, ub, rb of (p', u', rho') a reverse step forms, in order:
//   eos:  pbar = pb + w p' (recorded steps),  rbt = (c0^2 + 2 nl rho) pbar,
//         T0 = ta pbar, T1 = tb pbar           (then T0 <- A T0, T1 <- B T1 spectrally)
//   den:  R_xi = rb_xi + rbt + T1,  rb_xi <- R_xi q^2 / den_xi,
//         dbar_xi = -R_xi (q dt rho0 + 2 dt rho_xi') / den_xi + rho0 T0
//         + 2 dt R_xi src / den_xi at the source points (nonlinear); the
//         point's share coef sum_xi R_xi of dJ/ds_e(n), summed per element in
//         a fixed order (no floating-point atomics: the gradient is
//         repeatable bit for bit)
//   (spectral: T_xi = transpose-divergence of dbar_xi)
//   vel:  u = ub_xi + T_xi,  T_xi <- -q+ dt/rho0+ u,  ub_xi <- q+^2 u
//   (spectral: T_xi = transpose-gradient of T_xi)
//   sum:  pb = T0 + T1 + T2
// Each line is one x-row kernel: the inverse x transforms of its spectral
// inputs, the point-wise update, the forward x transforms of its spectral
// outputs (kw_adjx_eos, kw_adjx_den, kw_adjx_vel, kw_adjx_sum), as in the
// forward step's x passes.
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

// drive term of each source point in step n: coef_k s_e(n)
__global__ void __launch_bounds__(kThreads) kw_adj_src_add(SourceDev src, AdjDev a, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_src) return;
    a.add[k] = a.src_coef[k] * drive_at(src, a.src_elem[k], n);
}

// dJ/ds_e(n) = sum over element e's points of coef_k (R_0 + R_1 + R_2)(k)
// (one block per element, points in the order of the element's list)
__global__ void __launch_bounds__(kThreads) kw_adj_src_sum(AdjDev a, int n) {
    __shared__ double part[kThreads];
    const int e = blockIdx.x;
    double acc = 0.0;
    for (int j = a.elem_ptr[e] + (int)threadIdx.x; j < a.elem_ptr[e + 1]; j += kThreads) {
        const int k = a.elem_pts[j];
        const float rsum = a.rsrc[k] + a.rsrc[a.n_src + k] + a.rsrc[2 * a.n_src + k];
        acc += (double)a.src_coef[k] * (double)rsum;
    }
    const double total = block_sum(acc, part);
    if (threadIdx.x == 0) a.dJds[(size_t)n * a.n_elem + e] = total;
}

// ---------------------------------------------------------------------------
// fused x-row passes
// ---------------------------------------------------------------------------

// pbar = pb + w p' (p' from its packed spectrum: c2r / nx) on this thread's
// elements of row b, and rbt = (c0^2 + 2 nl rho) pbar when RBT
template <class Eng, bool RBT>
__device__ __forceinline__ void adj_pbar(const XArgs &a, const AdjDev &ad, const float2 *p_spec,
                                         int loss, int b, bool ok, int t, const RowLds &lds,
                                         const float2 *tws, size_t xrow0, uint32_t xlane,
                                         float2 (&v)[Eng::E]) {
    constexpr int E = Eng::E;
    const int M = a.g.M;
    const int cupd = Eng::out_count(a.pi, t);
    if (loss) row_c2r<Eng>(a, p_spec, b, ok, t, lds, v, tws, tws + M);
    const float inx = 1.0f / (float)a.g.nx;
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                float2 pbar = ld2(ad.pb, i);
                if (loss) {
                    const float2 w = ld2(ad.w, i);
                    pbar.x += w.x * (v[m].x * inx);
                    pbar.y += w.y * (v[m].y * inx);
                }
                if constexpr (RBT) {
                    float2 c = coef2_at(a.m.c0sq, i);
                    if (a.m.nonlinear) {
                        const float2 nl = coef2_at(a.m.nl, i);
                        const float2 r0 = ld2(ad.rho[0], i), r1 = ld2(ad.rho[1], i),
                                     r2 = ld2(ad.rho[2], i);
                        c.x += 2.0f * nl.x * (r0.x + r1.x + r2.x);
                        c.y += 2.0f * nl.y * (r0.y + r1.y + r2.y);
                    }
                    pbar = make_float2(c.x * pbar.x, c.y * pbar.y);
                }
                v[m] = pbar;
            }
        }
    }
}

// eos (absorbing media): rbt stored; ta pbar and tb pbar transformed into
// Sout[0], Sout[1] for the absorption operators
template <class Eng>
__global__ void __launch_bounds__(512) kw_adjx_eos(XArgs a, AdjDev ad, const float2 *p_spec, int loss) {
    KW_XPROLOGUE
    float2 v[E], tb[E];
    adj_pbar<Eng, false>(a, ad, p_spec, loss, b, ok, t, lds, tws, xrow0, xlane, v);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                const float2 pbar = v[m];
                float2 c = coef2_at(a.m.c0sq, i);
                if (a.m.nonlinear) {
                    const float2 nl = coef2_at(a.m.nl, i);
                    const float2 r0 = ld2(ad.rho[0], i), r1 = ld2(ad.rho[1], i), r2 = ld2(ad.rho[2], i);
                    c.x += 2.0f * nl.x * (r0.x + r1.x + r2.x);
                    c.y += 2.0f * nl.y * (r0.y + r1.y + r2.y);
                }
                st2(ad.rbt, i, make_float2(c.x * pbar.x, c.y * pbar.y));
                const float2 ta = coef2_at(a.m.ta, i), tbc = coef2_at(a.m.tb, i);
                v[m] = make_float2(ta.x * pbar.x, ta.y * pbar.y);
                tb[m] = make_float2(tbc.x * pbar.x, tbc.y * pbar.y);
            }
        }
    }
    row_r2c<Eng>(a, a.Sout[0], b, ok, t, lds, v, tws, tws + M);
    row_r2c<Eng>(a, a.Sout[1], b, ok, t, lds, tb, tws, tws + M);
}

// den: ABS -- T0' and T1' from Sin[0], Sin[1] (after the absorption
// operators) and rbt from the eos pass; otherwise pbar and rbt are formed here.
// The three divergence adjoints go (r2c) to Sout[0..2].  Source points of a
// row are found through an LDS line of point numbers (-1 elsewhere).
template <class Eng, bool ABS>
__global__ void __launch_bounds__(512) kw_adjx_den(XArgs a, AdjDev ad, const float2 *p_spec, int loss) {
    KW_XPROLOGUE
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const float dt = a.g.dt;
    float2 base[E], dcom[E];          // rbt (+ T1') and rho0 T0' (ABS)
    if constexpr (ABS) {
        row_c2r<Eng>(a, a.Sin[0], b, ok, t, lds, dcom, tws, tws + M);
        row_c2r<Eng>(a, a.Sin[1], b, ok, t, lds, base, tws, tws + M);
        if (ok) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cupd) {
                    const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                    const float2 rbt = ld2(ad.rbt, i);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    base[m] = c_add(rbt, base[m]);
                    dcom[m] = make_float2(r0.x * dcom[m].x, r0.y * dcom[m].y);
                }
            }
        }
    } else {
        adj_pbar<Eng, true>(a, ad, p_spec, loss, b, ok, t, lds, tws, xrow0, xlane, base);
#pragma unroll
        for (int m = 0; m < E; ++m) dcom[m] = make_float2(0.0f, 0.0f);
    }
    // point numbers of this row's source points
    int *const smap = reinterpret_cast<int *>(sh + (size_t)a.tb * row_pitch(M)) + (size_t)b * nx;
    int beg = 0, end = 0;
    if (a.src.row_ptr && ok) {
        beg = a.src.row_ptr[rr];
        end = a.src.row_ptr[rr + 1];
    }
    const bool any_src = __syncthreads_or(end > beg);     // block-uniform
    if (any_src) {
        for (int x = t; x < nx; x += L) smap[x] = -1;
        __syncthreads();
        for (int e = beg + t; e < end; e += L) smap[a.src.xpos[e]] = e;
        __syncthreads();
    }
    const float qy = a.t.pml_y[iy], qz = a.t.pml_z[iz];
#pragma unroll 1
    for (int g = 0; g < 3; ++g) {
        // salt = 0, unknown to the compiler (see kw_xden)
        const int salt = g * a.zero;
        const int ts = t + salt;
        const RowLds ldg{sh, lds.base + salt, lds.wave};
        float *const rb = pick3(ad.rb, g);
        const float *const dfw = pick3(ad.dfw, g);
        const float *const rho = pick3(ad.rho, g);
        float2 v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = make_float2(0.0f, 0.0f);
        if (ok) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cupd) {
                    const int x = 2 * Eng::out_index(a.pi, ts, m);
                    const XPos i{xrow0 + 2 * (size_t)m * (Eng::out_step(a.pi) + salt),
                                 (uint32_t)(b * nx + 2 * ts) * 4u};
                    float2 q;
                    if (g == 0) q = make_float2(a.t.pml_x[x], a.t.pml_x[x + 1]);
                    else if (g == 1) q = make_float2(qy, qy);
                    else q = make_float2(qz, qz);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    const float2 R = c_add(ld2(rb, i), base[m]);
                    float2 den = make_float2(1.0f, 1.0f), db;
                    if (a.m.nonlinear) {
                        const float2 d = ld2(dfw, i), rn = ld2(rho, i);
                        den = make_float2(1.0f + 2.0f * dt * d.x, 1.0f + 2.0f * dt * d.y);
                        db.x = -R.x * (q.x * dt * r0.x + 2.0f * dt * rn.x) / den.x;
                        db.y = -R.y * (q.y * dt * r0.y + 2.0f * dt * rn.y) / den.y;
                    } else {
                        db.x = -R.x * q.x * dt * r0.x;
                        db.y = -R.y * q.y * dt * r0.y;
                    }
                    st2(rb, i, make_float2(R.x * q.x * q.x / den.x, R.y * q.y * q.y / den.y));
                    v[m] = c_add(db, dcom[m]);
                    if (any_src) {
                        const int k0 = smap[x], k1 = smap[x + 1];
                        if (k0 >= 0) {
                            ad.rsrc[(size_t)g * ad.n_src + k0] = R.x;
                            if (a.m.nonlinear) v[m].x += R.x * 2.0f * dt * ad.add[k0] / den.x;
                        }
                        if (k1 >= 0) {
                            ad.rsrc[(size_t)g * ad.n_src + k1] = R.y;
                            if (a.m.nonlinear) v[m].y += R.y * 2.0f * dt * ad.add[k1] / den.y;
                        }
                    }
                }
            }
        }
        row_r2c<Eng>(a, pick3(a.Sout, g), b, ok, ts, ldg, v, tws, tws + M, salt);
    }
}

// vel: component blockIdx.y; T_xi from Sin, the transposed velocity update,
// -q+ dt/rho0+ u to Sout
template <class Eng>
__global__ void __launch_bounds__(512) kw_adjx_vel(XArgs a, AdjDev ad) {
    KW_XPROLOGUE
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const int xi = blockIdx.y;
    float2 v[E];
    row_c2r<Eng>(a, pick3(a.Sin, xi), b, ok, t, lds, v, tws, tws + M);
    if (ok) {
        float *const ub = pick3(ad.ub, xi);
        const Coef dtr = xi == 0 ? a.m.dtr[0] : xi == 1 ? a.m.dtr[1] : a.m.dtr[2];
        const float qy = a.t.pml_sy[iy], qz = a.t.pml_sz[iz];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const int x = 2 * Eng::out_index(a.pi, t, m);
                const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                float2 q;
                if (xi == 0) q = make_float2(a.t.pml_sx[x], a.t.pml_sx[x + 1]);
                else if (xi == 1) q = make_float2(qy, qy);
                else q = make_float2(qz, qz);
                const float2 u = c_add(ld2(ub, i), v[m]);
                const float2 d = coef2_at(dtr, i);
                st2(ub, i, make_float2(q.x * q.x * u.x, q.y * q.y * u.y));
                v[m] = make_float2(-q.x * d.x * u.x, -q.y * d.y * u.y);
            }
        }
    }
    row_r2c<Eng>(a, pick3(a.Sout, xi), b, ok, t, lds, v, tws, tws + M);
}

// sum: pb = T0 + T1 + T2 (the three transposed-gradient outputs in Sin)
template <class Eng>
__global__ void __launch_bounds__(512) kw_adjx_sum(XArgs a, AdjDev ad) {
    KW_XPROLOGUE
    float2 acc[E], v[E];
    row_c2r<Eng>(a, a.Sin[0], b, ok, t, lds, acc, tws, tws + M);
    row_c2r<Eng>(a, a.Sin[1], b, ok, t, lds, v, tws, tws + M);
#pragma unroll
    for (int m = 0; m < E; ++m) acc[m] = c_add(acc[m], v[m]);
    row_c2r<Eng>(a, a.Sin[2], b, ok, t, lds, v, tws, tws + M);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cupd)
                st2(ad.pb, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane}, c_add(acc[m], v[m]));
    }
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

hipError_t launch_adj_src(hipStream_t s, const AdjDev &a, const SourceDev &src, int n) {
    if (a.n_src == 0) return hipSuccess;
    hipLaunchKernelGGL(kw_adj_src_add, dim3((a.n_src + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       s, src, a, n);
    return hipGetLastError();
}

hipError_t launch_adj_src_sum(hipStream_t s, const AdjDev &a, int n) {
    if (a.n_src == 0) return hipSuccess;
    hipLaunchKernelGGL(kw_adj_src_sum, dim3(a.n_elem), dim3(kThreads), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_adjx(hipStream_t s, int pass, const GridDev &g, const LaunchCfg &c,
                       const Tables &t, const Medium &m, const SourceDev &src, const AdjDev &ad,
                       const float2 *p_spec, bool loss, float2 *const *Sin, float2 *const *Sout) {
    XArgs a{};
    a.g = g;
    a.t = t;
    a.m = m;
    a.src = src;
    a.pf = c.px;
    a.pi = c.pxi;
    a.tb = c.tb_x;
    for (int i = 0; i < 3; ++i) {
        a.Sin[i] = Sin ? Sin[i] : nullptr;
        a.Sout[i] = Sout ? Sout[i] : nullptr;
    }
    const int L = loss ? 1 : 0;
    dim3 grid((g.rows + c.tb_x - 1) / c.tb_x, pass == ADJX_VEL ? 3 : 1);
    dim3 block(c.tb_x * c.px.L);
    const size_t lds = x_lds_bytes(g.M, g.nx, c.tb_x, pass == ADJX_DEN || pass == ADJX_DEN_ABS);
    switch (pass) {
    case ADJX_EOS:
        KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_adjx_eos<Eng>), grid, block, lds, s, a, ad, p_spec, L));
        break;
    case ADJX_DEN:
        KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_adjx_den<Eng, false>), grid, block, lds, s, a, ad, p_spec, L));
        break;
    case ADJX_DEN_ABS:
        KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_adjx_den<Eng, true>), grid, block, lds, s, a, ad, p_spec, L));
        break;
    case ADJX_VEL:
        KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_adjx_vel<Eng>), grid, block, lds, s, a, ad));
        break;
    default:
        KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_adjx_sum<Eng>), grid, block, lds, s, a, ad));
        break;
    }
    return hipGetLastError();
}

}  // namespace kw
