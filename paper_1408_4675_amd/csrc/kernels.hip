// HIP kernels of one k-space pseudospectral time step for gfx950.
//
// Data layout (all device arrays carved from the caller's workspace):
//   real fields   float[nz][ny][nx]              (x fastest)
//   spectra       float2[nz][ny][M], M = nx / 2  (packed half spectrum along x)
// The x transform of a real row produces nx/2 + 1 complex values of which the
// first (kx = 0) and last (Nyquist) are real; they are packed into one complex
// value X0 + i XN at column 0, so a spectrum row has exactly the byte size of a
// real row.  The y and z transforms are linear and carry the packed column
// along; the fused z kernel separates it again (launch_zpair) before applying
// the k-space operators, which differ between kx = 0 and the Nyquist column.
//
// One step (absorbing case; Section 3.4 ordering of six forward and eight
// inverse 3D transforms):
//   ypass fwd(S0)                 (+ step counter and drive values, block 0)
//   zfused grad  S0 -> S1 S2 S3   Eq. (4a) operator  i k kappa e^{+ik d/2} / N
//   ypass inv(S1 S2 S3)
//   xvel         S1..S3 -> u_xi   x c2r, Eq. (4b) with PML, x r2c of u -> S1..S3
//   ypass fwd(S1 S2 S3)
//   zfused div   S1..S3 -> S4..S6 Eq. (4c) operator  i k kappa e^{-ik d/2} / N
//   ypass inv(S4 S5 S6)
//   xden         S4..S6 -> rho_xi Eq. (4d) with PML, nonlinear denominator and
//                mass source; rho = sum rho_xi; x r2c of rho0 sum du, rho -> S1 S2
//   ypass fwd(S1 S2)
//   zfused abs   S1 S2 -> S4 S5   k^(y-2) / N and k^(y-1) / N, Eq. (8)
//   ypass inv(S4 S5)
//   xeos         S4 S5 rho -> p   Eq. (6) with L_d of Eq. (8); sensors; x r2c of p -> S0
// Without absorption xden evaluates Eq. (6) itself and the last four kernels
// are skipped (four transforms fewer).
#include <hip/hip_runtime.h>
#include <float.h>
#include <limits.h>

#include "fft_dev.h"
#include "kw_internal.h"

namespace kw {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float coef_at(const Coef &c, size_t i) {
    return c.map ? c.map[i] : c.scalar;
}
__device__ __forceinline__ float2 coef2_at(const Coef &c, size_t i) {
    if (c.map) return *reinterpret_cast<const float2 *>(c.map + i);
    return make_float2(c.scalar, c.scalar);
}
__device__ __forceinline__ float2 ld2(const float *p, size_t i) {
    return *reinterpret_cast<const float2 *>(p + i);
}
__device__ __forceinline__ void st2(float *p, size_t i, float2 v) {
    *reinterpret_cast<float2 *>(p + i) = v;
}
// select one of three pointers without indexing the argument array at run time
template <class T>
__device__ __forceinline__ T pick3v(T p0, T p1, T p2, int i) {
    return i == 0 ? p0 : (i == 1 ? p1 : p2);
}
#define pick3(arr, i) pick3v((arr)[0], (arr)[1], (arr)[2], (i))
__device__ __forceinline__ float kappa_of(float k, float half_cdt) {
    const float x = half_cdt * k;
    return (x < 1.0e-3f) ? 1.0f - x * x * (1.0f / 6.0f) : sinf(x) / x;
}

// ---------------------------------------------------------------------------
// y pass: in-place column FFTs of up to three spectra
// ---------------------------------------------------------------------------
struct YArgs {
    float2 *f[3];
    int M, ny;
    FftPlan plan;
    const float2 *tw;
    int tb;
    // prologue (first kernel of a step): advance the step counter and
    // evaluate the drive value of every source element at t = (n + 1/2) dt
    int prologue;
    Counters cnt;
    SourceDev src;
};

template <int RM, bool INV>
__global__ void __launch_bounds__(512) kw_ypass(YArgs a) {
    extern __shared__ float2 sh[];
    const int tid = threadIdx.x;
    const int b = tid % a.tb, t = tid / a.tb;
    const int col = blockIdx.x * a.tb + b;
    const bool ok = col < a.M;
    float2 *base = pick3(a.f, (int)blockIdx.z) + (size_t)blockIdx.y * a.ny * a.M + col;
    const size_t stride = a.M;

    if (a.prologue && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) {
        const int n = *a.cnt.step;
        __syncthreads();
        if (tid == 0) *a.cnt.step = n + 1;
        for (int e = tid; e < a.src.n_elements; e += blockDim.x) {
            float s;
            if (a.src.signal) {
                s = (n < a.src.n_samples) ? a.src.signal[(size_t)e * a.src.n_samples + n] : 0.0f;
            } else {
                const double th = a.src.omega_dt * ((double)n + 0.5);
                s = (float)(a.src.amp_cos[e] * sin(th) + a.src.amp_sin[e] * cos(th));
            }
            a.src.drive[e] = s;
        }
    }

    float2 v[RM];
    const int R0 = a.plan.radix[0], nb0 = a.ny / R0;
    if (ok && t < nb0) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (r < R0) v[r] = base[(size_t)(t + r * nb0) * stride];
    }
    fft_run<INV, RM>(a.plan, a.tw, t, ColLds{sh, a.tb, b}, v);
    const int Rl = a.plan.radix[a.plan.np - 1], nbl = a.ny / Rl;
    if (ok && t < nbl) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (r < Rl) base[(size_t)(t + r * nbl) * stride] = v[r];
    }
}

// ---------------------------------------------------------------------------
// fused z pass: forward z FFT -> k-space operator(s) -> inverse z FFT
// ---------------------------------------------------------------------------
enum { ZM_GRAD = 0, ZM_DIV = 1, ZM_ABS = 2 };

struct ZArgs {
    const float2 *in[3];
    float2 *out[3];
    GridDev g;
    Tables t;
    FftPlan pf, pi;          // forward plan and its reverse
    int tb;
};

// multiplier of output o at (kx index ix (M = Nyquist), ky index iy, kz index iz)
template <int MODE>
__device__ __forceinline__ float2 z_operator(const ZArgs &a, int o, int ix, int iy, int iz) {
    const float kx = a.t.kx[ix], ky = a.t.ky[iy], kz = a.t.kz[iz];
    const float k2 = kx * kx + ky * ky + kz * kz;
    if constexpr (MODE == ZM_ABS) {
        if (k2 <= 0.0f) return make_float2(0.0f, 0.0f);
        const float e = (o == 0) ? a.g.y_tau : a.g.y_eta;
        return make_float2(exp2f(e * log2f(k2)) * a.g.inv_n, 0.0f);
    } else {
        const float s = kappa_of(sqrtf(k2), a.g.half_cdt) * a.g.inv_n;
        float2 d;
        if (MODE == ZM_GRAD)
            d = (o == 0) ? a.t.dpx[ix] : (o == 1) ? a.t.dpy[iy] : a.t.dpz[iz];
        else
            d = (o == 0) ? a.t.dmx[ix] : (o == 1) ? a.t.dmy[iy] : a.t.dmz[iz];
        return c_scale(d, s);
    }
}

template <int RM, int MODE>
__global__ void __launch_bounds__(512) kw_zfused(ZArgs a) {
    extern __shared__ float2 sh[];
    const int tid = threadIdx.x;
    const int b = tid % a.tb, t = tid / a.tb;
    const int col = blockIdx.x * a.tb + b;
    const int iy = blockIdx.y;
    const bool ok = col < a.g.M;
    const int ix = ok ? col : 0;
    const size_t off = (size_t)iy * a.g.M + col;
    const size_t stride = (size_t)a.g.M * a.g.ny;
    const int nz = a.g.nz;
    const ColLds lds{sh, a.tb, b};
    const int R0 = a.pf.radix[0], nb0 = nz / R0;
    const int Rl = a.pf.radix[a.pf.np - 1], nbl = nz / Rl;
    constexpr int NIN = (MODE == ZM_GRAD) ? 1 : (MODE == ZM_DIV) ? 3 : 2;

#pragma unroll 1
    for (int f = 0; f < NIN; ++f) {
        float2 v[RM];
        if (ok && t < nb0) {
            const float2 *src = pick3(a.in, f) + off;
#pragma unroll
            for (int r = 0; r < RM; ++r)
                if (r < R0) v[r] = src[(size_t)(t + r * nb0) * stride];
        }
        fft_run<false, RM>(a.pf, a.t.tw_z, t, lds, v);
        if constexpr (MODE == ZM_GRAD) {
            float2 vf[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) vf[r] = v[r];
#pragma unroll 1
            for (int o = 0; o < 3; ++o) {
                if (t < nbl) {
#pragma unroll
                    for (int r = 0; r < RM; ++r)
                        if (r < Rl) v[r] = c_mul(vf[r], z_operator<MODE>(a, o, ix, iy, t + r * nbl));
                }
                fft_run<true, RM>(a.pi, a.t.tw_z, t, lds, v);
                if (ok && t < nb0) {
                    float2 *dst = pick3(a.out, o) + off;
#pragma unroll
                    for (int r = 0; r < RM; ++r)
                        if (r < R0) dst[(size_t)(t + r * nb0) * stride] = v[r];
                }
            }
        } else {
            if (t < nbl) {
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (r < Rl) v[r] = c_mul(v[r], z_operator<MODE>(a, f, ix, iy, t + r * nbl));
            }
            fft_run<true, RM>(a.pi, a.t.tw_z, t, lds, v);
            if (ok && t < nb0) {
                float2 *dst = pick3(a.out, f) + off;
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (r < R0) dst[(size_t)(t + r * nb0) * stride] = v[r];
            }
        }
    }
}

// Column kx = 0 holds X0 + i XN (X0: kx = 0 part, XN: Nyquist part; both real
// before the y/z transforms).  After the forward z transform the two parts are
// separated with the conjugate-symmetric partner at (-ky, -kz):
//   A = (C(ky,kz) + conj C(-ky,-kz)) / 2,   B = (C(ky,kz) - conj C(-ky,-kz)) / 2i
// each gets its own operator, and the results are repacked as A' + i B'.  A
// block handles the rows ky and -ky (b = 0, 1) of column 0.
template <int RM, int MODE>
__global__ void __launch_bounds__(512) kw_zpair(ZArgs a) {
    extern __shared__ float2 sh[];
    const int tid = threadIdx.x;
    const int b = tid & 1, t = tid >> 1;
    const int ny = a.g.ny, nz = a.g.nz;
    const int ky0 = blockIdx.x;
    const int ky1 = (ny - ky0) % ny;
    const int iy = b ? ky1 : ky0;
    const bool store = (b == 0) || (ky1 != ky0);
    const size_t off = (size_t)iy * a.g.M;   // column 0
    const size_t stride = (size_t)a.g.M * ny;
    const ColLds lds{sh, 2, b};
    const int R0 = a.pf.radix[0], nb0 = nz / R0;
    const int Rl = a.pf.radix[a.pf.np - 1], nbl = nz / Rl;
    constexpr int NIN = (MODE == ZM_GRAD) ? 1 : (MODE == ZM_DIV) ? 3 : 2;
    const int M = a.g.M;

#pragma unroll 1
    for (int f = 0; f < NIN; ++f) {
        float2 v[RM];
        if (t < nb0) {
            const float2 *src = pick3(a.in, f) + off;
#pragma unroll
            for (int r = 0; r < RM; ++r)
                if (r < R0) v[r] = src[(size_t)(t + r * nb0) * stride];
        }
        fft_run<false, RM>(a.pf, a.t.tw_z, t, lds, v);
        // publish both columns' spectra, then read the partner values
        if (t < nbl) {
#pragma unroll
            for (int r = 0; r < RM; ++r)
                if (r < Rl) lds.st(t + r * nbl, v[r]);
        }
        __syncthreads();
        float2 va[RM], vb[RM];
        if (t < nbl) {
            const ColLds other{sh, 2, 1 - b};
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                if (r < Rl) {
                    const int iz = t + r * nbl;
                    const float2 c = v[r];
                    const float2 pc = c_conj(other.ld((nz - iz) % nz));
                    va[r] = c_scale(c_add(c, pc), 0.5f);
                    // (c - pc) / (2i) = -i (c - pc) / 2
                    const float2 d = c_sub(c, pc);
                    vb[r] = make_float2(0.5f * d.y, -0.5f * d.x);
                }
            }
        }
        __syncthreads();
        const int no = (MODE == ZM_GRAD) ? 3 : 1;
#pragma unroll 1
        for (int oo = 0; oo < no; ++oo) {
            const int o = (MODE == ZM_GRAD) ? oo : f;
            if (t < nbl) {
#pragma unroll
                for (int r = 0; r < RM; ++r) {
                    if (r < Rl) {
                        const int iz = t + r * nbl;
                        const float2 ya = c_mul(va[r], z_operator<MODE>(a, o, 0, iy, iz));
                        const float2 yb = c_mul(vb[r], z_operator<MODE>(a, o, M, iy, iz));
                        v[r] = make_float2(ya.x - yb.y, ya.y + yb.x);   // ya + i yb
                    }
                }
            }
            fft_run<true, RM>(a.pi, a.t.tw_z, t, lds, v);
            if (store && t < nb0) {
                float2 *dst = pick3(a.out, o) + off;
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    if (r < R0) dst[(size_t)(t + r * nb0) * stride] = v[r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// x passes: rows of the real grid, fused with the element-wise updates
// ---------------------------------------------------------------------------
struct XArgs {
    GridDev g;
    Tables t;
    Medium m;
    SourceDev src;
    SensorDev sen;
    Counters cnt;
    FftPlan pf, pi;          // forward plan (length M) and its reverse
    int tb;                  // rows per block
    const float2 *Sin[3];
    float2 *Sout[3];
    float *fld[3];           // u or rho components
    float *rho_total;
    const float *rsrc;       // xfwd: real input
    float *rdst;             // xinv: real output
    float scale;
};

// c2r: packed spectrum row -> v[r] = x[2n] + i x[2n+1], n = t + r M/R0
// (unnormalised; the result is nx times the inverse DFT)
template <int RM>
__device__ __forceinline__ void row_c2r(const XArgs &a, const float2 *__restrict__ row, bool ok,
                                        int t, const RowLds &lds, float2 (&v)[RM]) {
    const int M = a.g.M;
    const int Ra = a.pi.radix[0], nba = M / Ra;
    if (ok && t < nba) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (r < Ra) {
                const int k = t + r * nba;
                const float2 P = row[k];
                float2 xk, xm;
                if (k == 0) {
                    xk = make_float2(P.x, 0.0f);
                    xm = make_float2(P.y, 0.0f);
                } else {
                    xk = P;
                    xm = row[M - k];
                }
                const float2 A = make_float2(xk.x + xm.x, xk.y - xm.y);        // xk + conj(xm)
                const float2 D = make_float2(xk.x - xm.x, xk.y + xm.y);        // xk - conj(xm)
                const float2 B = c_mulc(D, a.t.tw_post[k]);                     // * w^-k
                v[r] = make_float2(A.x - B.y, A.y + B.x);                       // A + i B
            }
        }
    }
    fft_run<true, RM>(a.pi, a.t.tw_x, t, lds, v);
}

// r2c: v[r] = x[2n] + i x[2n+1], n = t + r M/R0  ->  packed spectrum row
template <int RM>
__device__ __forceinline__ void row_r2c(const XArgs &a, float2 *__restrict__ row, bool ok, int t,
                                        const RowLds &lds, float2 (&v)[RM]) {
    const int M = a.g.M;
    fft_run<false, RM>(a.pf, a.t.tw_x, t, lds, v);
    const int Rl = a.pf.radix[a.pf.np - 1], nbl = M / Rl;
    if (t < nbl) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (r < Rl) lds.st(t + r * nbl, v[r]);
    }
    __syncthreads();
    if (ok && t < nbl) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (r < Rl) {
                const int k = t + r * nbl;
                const float2 Z = v[r];
                float2 out;
                if (k == 0) {
                    out = make_float2(Z.x + Z.y, Z.x - Z.y);     // X0 + i XN
                } else {
                    const float2 Zm = c_conj(lds.ld(M - k));
                    const float2 A = c_scale(c_add(Z, Zm), 0.5f);
                    const float2 Bh = c_scale(c_sub(Z, Zm), 0.5f);
                    const float2 c = c_mul(a.t.tw_post[k], Bh);
                    out = make_float2(A.x + c.y, A.y - c.x);     // A - i w^k B
                }
                row[k] = out;
            }
        }
    }
    __syncthreads();
}

template <int RM>
__global__ void __launch_bounds__(512) kw_xvel(XArgs a) {
    extern __shared__ float2 sh[];
    const int L = a.pf.L;
    const int tid = threadIdx.x, t = tid % L, b = tid / L;
    const int row = blockIdx.x * a.tb + b;
    const bool ok = row < a.g.rows;
    const int rr = ok ? row : 0;
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const int M = a.g.M, nx = a.g.nx;
    const RowLds lds{sh, b * row_pitch(M)};
    const int R0 = a.pf.radix[0], nb0 = M / R0;
    const size_t rbase = (size_t)rr * nx;

#pragma unroll 1
    for (int xi = 0; xi < 3; ++xi) {
        float2 v[RM];
        row_c2r<RM>(a, pick3(a.Sin, xi) + (size_t)rr * M, ok, t, lds, v);
        if (ok && t < nb0) {
            float *u = pick3(a.fld, xi);
            const Coef dtr = xi == 0 ? a.m.dtr[0] : xi == 1 ? a.m.dtr[1] : a.m.dtr[2];
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                if (r < R0) {
                    const int x = 2 * (t + r * nb0);
                    const size_t i = rbase + x;
                    float2 q;
                    if (xi == 0) q = make_float2(a.t.pml_sx[x], a.t.pml_sx[x + 1]);
                    else if (xi == 1) q = make_float2(a.t.pml_sy[iy], a.t.pml_sy[iy]);
                    else q = make_float2(a.t.pml_sz[iz], a.t.pml_sz[iz]);
                    const float2 d = coef2_at(dtr, i);
                    const float2 u0 = ld2(u, i);
                    const float2 g = v[r];
                    float2 un;
                    un.x = q.x * (q.x * u0.x - d.x * g.x);
                    un.y = q.y * (q.y * u0.y - d.y * g.y);
                    st2(u, i, un);
                    v[r] = un;
                }
            }
        }
        row_r2c<RM>(a, pick3(a.Sout, xi) + (size_t)rr * M, ok, t, lds, v);
    }
}

// Source values of the rows of this block, scattered into a per-row LDS line
// of nx floats (zero where there is no source point).  Returns whether the
// block has any source point (uniform over the block).
__device__ __forceinline__ bool scatter_source(const XArgs &a, float *line, int row, bool ok,
                                               int t, int L, int b) {
    const int nx = a.g.nx;
    int beg = 0, end = 0;
    if (a.src.row_ptr && ok) {
        beg = a.src.row_ptr[row];
        end = a.src.row_ptr[row + 1];
    }
    const bool any = __syncthreads_or(end > beg);
    if (!any) return false;
    float *mine = line + (size_t)b * nx;
    for (int x = t; x < nx; x += L) mine[x] = 0.0f;
    __syncthreads();
    for (int e = beg + t; e < end; e += L)
        mine[a.src.xpos[e]] = a.src.coef[e] * a.src.drive[a.src.elem[e]];
    __syncthreads();
    return true;
}

// Pressure of the rows of this block at the sensor points (mask mode).
template <int RM>
__device__ __forceinline__ void record_mask(const XArgs &a, float *line, int row, bool ok, int t,
                                            int L, int b, int step, const float2 (&p)[RM], int R0,
                                            int nb0) {
    const int nx = a.g.nx;
    int beg = 0, end = 0;
    if (ok) {
        beg = a.sen.row_ptr[row];
        end = a.sen.row_ptr[row + 1];
    }
    const bool any = __syncthreads_or(end > beg);
    if (!any) return;
    float *mine = line + (size_t)b * nx;
    if (ok && t < nb0) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (r < R0) {
                const int x = 2 * (t + r * nb0);
                mine[x] = p[r].x;
                mine[x + 1] = p[r].y;
            }
        }
    }
    __syncthreads();
    const int slot = step - a.sen.record_start;
    for (int e = beg + t; e < end; e += L) {
        const int id = a.sen.sid[e];
        const float pv = mine[a.sen.xpos[e]];
        if (a.sen.p_max) a.sen.p_max[id] = fmaxf(a.sen.p_max[id], pv);
        if (a.sen.p_sum2) a.sen.p_sum2[id] += pv * pv;
        if (a.sen.series && slot < a.sen.capacity)
            a.sen.series[(size_t)slot * a.sen.n_points + id] = pv;
    }
    __syncthreads();
}

// equation of state, sensors and x r2c of the new pressure (v holds p)
template <int RM>
__device__ __forceinline__ void finish_pressure(const XArgs &a, float *line, int row, bool ok,
                                                int t, int L, int b, const RowLds &lds,
                                                float2 (&v)[RM]) {
    const int M = a.g.M, nx = a.g.nx;
    const int R0 = a.pf.radix[0], nb0 = M / R0;
    const size_t rbase = (size_t)(ok ? row : 0) * nx;
    const int step = *a.cnt.step;
    const bool rec = step >= a.sen.record_start;
    bool bad = false;
    if (ok && t < nb0) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (r < R0) {
                const float2 p = v[r];
                bad |= !(__builtin_isfinite(p.x) && __builtin_isfinite(p.y));
                if (rec && a.sen.all_points) {
                    const size_t i = rbase + 2 * (t + r * nb0);
                    if (a.sen.p_max) {
                        const float2 m = ld2(a.sen.p_max, i);
                        st2(a.sen.p_max, i, make_float2(fmaxf(m.x, p.x), fmaxf(m.y, p.y)));
                    }
                    if (a.sen.p_sum2) {
                        const float2 s = ld2(a.sen.p_sum2, i);
                        st2(a.sen.p_sum2, i, make_float2(s.x + p.x * p.x, s.y + p.y * p.y));
                    }
                }
            }
        }
    }
    if (bad) atomicMin(a.cnt.nonfinite, step);
    if (rec && !a.sen.all_points && a.sen.row_ptr)
        record_mask<RM>(a, line, row, ok, t, L, b, step, v, R0, nb0);
    row_r2c<RM>(a, a.Sout[0] + (size_t)(ok ? row : 0) * M, ok, t, lds, v);
}

template <int RM>
__global__ void __launch_bounds__(512) kw_xden(XArgs a) {
    extern __shared__ float2 sh[];
    const int L = a.pf.L;
    const int tid = threadIdx.x, t = tid % L, b = tid / L;
    const int row = blockIdx.x * a.tb + b;
    const bool ok = row < a.g.rows;
    const int rr = ok ? row : 0;
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const int M = a.g.M, nx = a.g.nx;
    const RowLds lds{sh, b * row_pitch(M)};
    float *line = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M));
    const int R0 = a.pf.radix[0], nb0 = M / R0;
    const size_t rbase = (size_t)rr * nx;
    const float dt = a.g.dt;

    const bool has_src = scatter_source(a, line, rr, ok, t, L, b);
    const float *mysrc = line + (size_t)b * nx;

    float2 acc_rho[RM], acc_div[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) acc_rho[r] = acc_div[r] = make_float2(0.0f, 0.0f);

#pragma unroll 1
    for (int xi = 0; xi < 3; ++xi) {
        float2 v[RM];
        row_c2r<RM>(a, pick3(a.Sin, xi) + (size_t)rr * M, ok, t, lds, v);
        if (ok && t < nb0) {
            float *rho = pick3(a.fld, xi);
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                if (r < R0) {
                    const int x = 2 * (t + r * nb0);
                    const size_t i = rbase + x;
                    float2 q;
                    if (xi == 0) q = make_float2(a.t.pml_x[x], a.t.pml_x[x + 1]);
                    else if (xi == 1) q = make_float2(a.t.pml_y[iy], a.t.pml_y[iy]);
                    else q = make_float2(a.t.pml_z[iz], a.t.pml_z[iz]);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    const float2 d = v[r];
                    const float2 old = ld2(rho, i);
                    float2 nw;
                    nw.x = q.x * (q.x * old.x - dt * r0.x * d.x);
                    nw.y = q.y * (q.y * old.y - dt * r0.y * d.y);
                    if (a.m.nonlinear) {
                        nw.x = nw.x / (1.0f + 2.0f * dt * d.x);
                        nw.y = nw.y / (1.0f + 2.0f * dt * d.y);
                    }
                    if (has_src) {
                        nw.x += mysrc[x];
                        nw.y += mysrc[x + 1];
                    }
                    st2(rho, i, nw);
                    acc_rho[r] = c_add(acc_rho[r], nw);
                    acc_div[r] = c_add(acc_div[r], d);
                }
            }
        }
    }

    float2 v[RM];
    if (a.m.absorbing) {
        // store rho = sum rho_xi for the equation of state, transform rho0 sum du and rho
        if (ok && t < nb0) {
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                if (r < R0) {
                    const size_t i = rbase + 2 * (t + r * nb0);
                    st2(a.rho_total, i, acc_rho[r]);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    v[r] = make_float2(r0.x * acc_div[r].x, r0.y * acc_div[r].y);
                }
            }
        }
        row_r2c<RM>(a, a.Sout[0] + (size_t)rr * M, ok, t, lds, v);
#pragma unroll
        for (int r = 0; r < RM; ++r) v[r] = acc_rho[r];
        row_r2c<RM>(a, a.Sout[1] + (size_t)rr * M, ok, t, lds, v);
    } else {
        if (ok && t < nb0) {
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                if (r < R0) {
                    const size_t i = rbase + 2 * (t + r * nb0);
                    const float2 rho = acc_rho[r];
                    const float2 c2 = coef2_at(a.m.c0sq, i);
                    float2 p = make_float2(c2.x * rho.x, c2.y * rho.y);
                    if (a.m.nonlinear) {
                        const float2 nl = coef2_at(a.m.nl, i);
                        p.x += nl.x * rho.x * rho.x;
                        p.y += nl.y * rho.y * rho.y;
                    }
                    v[r] = p;
                }
            }
        }
        finish_pressure<RM>(a, line, rr, ok, t, L, b, lds, v);
    }
}

template <int RM>
__global__ void __launch_bounds__(512) kw_xeos(XArgs a) {
    extern __shared__ float2 sh[];
    const int L = a.pf.L;
    const int tid = threadIdx.x, t = tid % L, b = tid / L;
    const int row = blockIdx.x * a.tb + b;
    const bool ok = row < a.g.rows;
    const int rr = ok ? row : 0;
    const int M = a.g.M, nx = a.g.nx;
    const RowLds lds{sh, b * row_pitch(M)};
    float *line = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M));
    const int R0 = a.pf.radix[0], nb0 = M / R0;
    const size_t rbase = (size_t)rr * nx;

    float2 va[RM], v[RM];
    row_c2r<RM>(a, a.Sin[0] + (size_t)rr * M, ok, t, lds, va);
    row_c2r<RM>(a, a.Sin[1] + (size_t)rr * M, ok, t, lds, v);
    if (ok && t < nb0) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            if (r < R0) {
                const size_t i = rbase + 2 * (t + r * nb0);
                const float2 rho = ld2(a.rho_total, i);
                const float2 c2 = coef2_at(a.m.c0sq, i);
                const float2 ta = coef2_at(a.m.ta, i);
                const float2 tb = coef2_at(a.m.tb, i);
                float2 p;
                p.x = c2.x * rho.x + ta.x * va[r].x + tb.x * v[r].x;
                p.y = c2.y * rho.y + ta.y * va[r].y + tb.y * v[r].y;
                if (a.m.nonlinear) {
                    const float2 nl = coef2_at(a.m.nl, i);
                    p.x += nl.x * rho.x * rho.x;
                    p.y += nl.y * rho.y * rho.y;
                }
                v[r] = p;
            }
        }
    }
    finish_pressure<RM>(a, line, rr, ok, t, L, b, lds, v);
}

template <int RM>
__global__ void __launch_bounds__(512) kw_xfwd(XArgs a) {
    extern __shared__ float2 sh[];
    const int L = a.pf.L;
    const int tid = threadIdx.x, t = tid % L, b = tid / L;
    const int row = blockIdx.x * a.tb + b;
    const bool ok = row < a.g.rows;
    const int rr = ok ? row : 0;
    const int M = a.g.M;
    const RowLds lds{sh, b * row_pitch(M)};
    const int R0 = a.pf.radix[0], nb0 = M / R0;
    float2 v[RM];
    if (ok && t < nb0) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (r < R0) v[r] = ld2(a.rsrc, (size_t)rr * a.g.nx + 2 * (t + r * nb0));
    }
    row_r2c<RM>(a, a.Sout[0] + (size_t)rr * M, ok, t, lds, v);
}

template <int RM>
__global__ void __launch_bounds__(512) kw_xinv(XArgs a) {
    extern __shared__ float2 sh[];
    const int L = a.pf.L;
    const int tid = threadIdx.x, t = tid % L, b = tid / L;
    const int row = blockIdx.x * a.tb + b;
    const bool ok = row < a.g.rows;
    const int rr = ok ? row : 0;
    const int M = a.g.M;
    const RowLds lds{sh, b * row_pitch(M)};
    const int R0 = a.pf.radix[0], nb0 = M / R0;
    float2 v[RM];
    row_c2r<RM>(a, a.Sin[0] + (size_t)rr * M, ok, t, lds, v);
    if (ok && t < nb0) {
#pragma unroll
        for (int r = 0; r < RM; ++r)
            if (r < R0)
                st2(a.rdst, (size_t)rr * a.g.nx + 2 * (t + r * nb0), c_scale(v[r], a.scale));
    }
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void kw_fill(float *p, size_t n, float v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int rm_for(const FftPlan &a, const FftPlan &b) {
    return (a.rmax > 16 || b.rmax > 16) ? 32 : 16;
}

hipError_t launch_ypass(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                        float2 *const *fields, int nfields, bool inverse,
                        const Counters *prologue, const SourceDev *src) {
    YArgs a{};
    for (int i = 0; i < nfields; ++i) a.f[i] = fields[i];
    a.M = g.M;
    a.ny = g.ny;
    a.plan = inverse ? c.pyi : c.py;
    a.tw = t.tw_y;
    a.tb = c.tb_y;
    a.prologue = prologue != nullptr;
    if (prologue) a.cnt = *prologue;
    if (src) a.src = *src;
    dim3 grid((g.M + a.tb - 1) / a.tb, g.nz, nfields);
    dim3 block(a.tb * a.plan.L);
    size_t lds = (size_t)a.tb * g.ny * sizeof(float2);
    const int rm = rm_for(c.py, c.pyi);
    if (rm == 16) {
        if (inverse) hipLaunchKernelGGL((kw_ypass<16, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((kw_ypass<16, false>), grid, block, lds, s, a);
    } else {
        if (inverse) hipLaunchKernelGGL((kw_ypass<32, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((kw_ypass<32, false>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

template <int RM>
static void zfused_dispatch(int mode, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                            const ZArgs &a) {
    if (mode == ZM_GRAD) hipLaunchKernelGGL((kw_zfused<RM, ZM_GRAD>), grid, block, lds, s, a);
    else if (mode == ZM_DIV) hipLaunchKernelGGL((kw_zfused<RM, ZM_DIV>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((kw_zfused<RM, ZM_ABS>), grid, block, lds, s, a);
}
template <int RM>
static void zpair_dispatch(int mode, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                           const ZArgs &a) {
    if (mode == ZM_GRAD) hipLaunchKernelGGL((kw_zpair<RM, ZM_GRAD>), grid, block, lds, s, a);
    else if (mode == ZM_DIV) hipLaunchKernelGGL((kw_zpair<RM, ZM_DIV>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((kw_zpair<RM, ZM_ABS>), grid, block, lds, s, a);
}

static ZArgs make_zargs(const GridDev &g, const LaunchCfg &c, const Tables &t, int mode,
                        float2 *const *in, float2 *const *out) {
    ZArgs a{};
    const int nin = (mode == ZM_GRAD) ? 1 : (mode == ZM_DIV) ? 3 : 2;
    const int nout = (mode == ZM_ABS) ? 2 : 3;
    for (int i = 0; i < nin; ++i) a.in[i] = in[i];
    for (int i = 0; i < nout; ++i) a.out[i] = out[i];
    a.g = g;
    a.t = t;
    a.pf = c.pz;
    a.pi = c.pzi;
    return a;
}

hipError_t launch_zfused(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                         int mode, float2 *const *in, float2 *const *out, int) {
    ZArgs a = make_zargs(g, c, t, mode, in, out);
    a.tb = c.tb_z;
    dim3 grid((g.M + a.tb - 1) / a.tb, g.ny);
    dim3 block(a.tb * c.pz.L);
    size_t lds = (size_t)a.tb * g.nz * sizeof(float2);
    if (rm_for(c.pz, c.pzi) == 16) zfused_dispatch<16>(mode, grid, block, lds, s, a);
    else zfused_dispatch<32>(mode, grid, block, lds, s, a);
    return hipGetLastError();
}

hipError_t launch_zpair(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                        int mode, float2 *const *in, float2 *const *out) {
    ZArgs a = make_zargs(g, c, t, mode, in, out);
    a.tb = 2;
    dim3 grid(g.ny / 2 + 1);
    dim3 block(2 * c.pz.L);
    size_t lds = (size_t)2 * g.nz * sizeof(float2);
    if (rm_for(c.pz, c.pzi) == 16) zpair_dispatch<16>(mode, grid, block, lds, s, a);
    else zpair_dispatch<32>(mode, grid, block, lds, s, a);
    return hipGetLastError();
}

static XArgs make_xargs(const GridDev &g, const LaunchCfg &c, const Tables &t) {
    XArgs a{};
    a.g = g;
    a.t = t;
    a.pf = c.px;
    a.pi = c.pxi;
    a.tb = c.tb_x;
    return a;
}
static inline size_t x_lds(const GridDev &g, const LaunchCfg &c, bool line) {
    size_t n = (size_t)c.tb_x * row_pitch(g.M) * sizeof(float2);
    if (line) n += (size_t)c.tb_x * g.nx * sizeof(float);
    return n;
}
#define KW_XLAUNCH(KERNEL, LINE)                                                         \
    do {                                                                                 \
        dim3 grid((g.rows + c.tb_x - 1) / c.tb_x);                                       \
        dim3 block(c.tb_x * c.px.L);                                                     \
        size_t lds = x_lds(g, c, LINE);                                                  \
        if (rm_for(c.px, c.pxi) == 16) hipLaunchKernelGGL((KERNEL<16>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((KERNEL<32>), grid, block, lds, s, a);                   \
    } while (0)

hipError_t launch_xvel(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, float2 *const *S, float *const *u) {
    XArgs a = make_xargs(g, c, t);
    a.m = m;
    for (int i = 0; i < 3; ++i) {
        a.Sin[i] = S[i];
        a.Sout[i] = S[i];
        a.fld[i] = u[i];
    }
    KW_XLAUNCH(kw_xvel, false);
    return hipGetLastError();
}

hipError_t launch_xden(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, const SourceDev &src, const SensorDev &sen,
                       const Counters &cnt, float2 *const *Sin, float *const *rho,
                       float *rho_total, float2 *const *Sout) {
    XArgs a = make_xargs(g, c, t);
    a.m = m;
    a.src = src;
    a.sen = sen;
    a.cnt = cnt;
    for (int i = 0; i < 3; ++i) {
        a.Sin[i] = Sin[i];
        a.fld[i] = rho[i];
    }
    a.Sout[0] = Sout[0];
    a.Sout[1] = Sout[1];
    a.rho_total = rho_total;
    KW_XLAUNCH(kw_xden, true);
    return hipGetLastError();
}

hipError_t launch_xeos(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, const SensorDev &sen, const Counters &cnt,
                       float2 *const *Sin, const float *rho_total, float2 *Sout) {
    XArgs a = make_xargs(g, c, t);
    a.m = m;
    a.sen = sen;
    a.cnt = cnt;
    a.Sin[0] = Sin[0];
    a.Sin[1] = Sin[1];
    a.rho_total = const_cast<float *>(rho_total);
    a.Sout[0] = Sout;
    KW_XLAUNCH(kw_xeos, true);
    return hipGetLastError();
}

hipError_t launch_xfwd(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const float *src, float2 *dst) {
    XArgs a = make_xargs(g, c, t);
    a.rsrc = src;
    a.Sout[0] = dst;
    KW_XLAUNCH(kw_xfwd, false);
    return hipGetLastError();
}

hipError_t launch_xinv(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const float2 *src, float *dst, float scale) {
    XArgs a = make_xargs(g, c, t);
    a.Sin[0] = src;
    a.rdst = dst;
    a.scale = scale;
    KW_XLAUNCH(kw_xinv, false);
    return hipGetLastError();
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
