// HIP kernels of one k-space pseudospectral time step for gfx950 (templates;
// instantiated by the launcher files kernels_yz.hip and kernels_x.hip).
//
// Data layout (all device arrays carved from the caller's workspace):
//   real fields   float[nz][ny][nx]              (x fastest)
//   spectra       float2[nz][ny][M], M = nx / 2  (packed half spectrum along x)
// The x transform of a real row produces nx/2 + 1 complex values of which the
// first (kx = 0) and last (Nyquist) are real; they are packed into one complex
// value X0 + i XN at column 0, so a spectrum row has exactly the byte size of a
// real row.  The y and z transforms are linear and carry the packed column
// along; the kw_zpair kernel separates it again for column 0 before
// applying the k-space operators, which differ between kx = 0 and Nyquist.
//
// One step (absorbing case; six forward and eight inverse 3D transforms, in
// the order of Section 3.4):
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
#pragma once

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
// select one of three values without indexing the argument array at run time
// (a run-time index into a by-value kernel argument forces it into scratch)
template <class T>
__device__ __forceinline__ T pick3v(T p0, T p1, T p2, int i) {
    return i == 0 ? p0 : (i == 1 ? p1 : p2);
}
#define pick3(arr, i) pick3v((arr)[0], (arr)[1], (arr)[2], (i))

// kappa = sinc(x) = sin(x)/x with x^2 = (c_ref dt / 2)^2 k^2, evaluated as its
// Taylor polynomial in x^2 up to x^16/17! (truncation error below 1e-9 for
// x <= 1.7, which covers every stable CFL number of the scheme); larger
// arguments take sinf(x)/x.  No sqrt and no range reduction on the common path.
__device__ __forceinline__ float kappa_of_x2(float x2) {
    if (x2 > 2.89f) {
        const float x = sqrtf(x2);
        return sinf(x) / x;
    }
    float p = 1.0f / 355687428096000.0f;            //  1/17!
    p = p * x2 - 1.0f / 1307674368000.0f;           // -1/15!
    p = p * x2 + 1.0f / 6227020800.0f;              //  1/13!
    p = p * x2 - 1.0f / 39916800.0f;                // -1/11!
    p = p * x2 + 1.0f / 362880.0f;                  //  1/9!
    p = p * x2 - 1.0f / 5040.0f;                    // -1/7!
    p = p * x2 + 1.0f / 120.0f;                     //  1/5!
    p = p * x2 - 1.0f / 6.0f;                       // -1/3!
    return p * x2 + 1.0f;
}

// ---------------------------------------------------------------------------
// y pass: in-place column FFTs of up to three spectra
// ---------------------------------------------------------------------------
struct YArgs {
    float2 *f[3];
    int M, ny;
    FftPlan plan;            // forward plan, or the reversed plan for the inverse
    const float2 *tw;
    int tb;
    // prologue (first kernel of a step): advance the step counter and
    // evaluate the drive value of every source element at t = (n + 1/2) dt
    int prologue;
    Counters cnt;
    SourceDev src;
};

template <class Eng, bool INV>
__global__ void __launch_bounds__(512) kw_ypass(YArgs a) {
    constexpr int E = Eng::E;
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

    float2 v[E];
    const int cin = Eng::in_count(a.plan, t);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = base[(size_t)Eng::in_index(a.plan, t, m) * stride];
    }
    Eng::template run<INV>(a.plan, a.tw, t, ColLds{sh, a.tb, b}, v);
    const int cout = Eng::out_count(a.plan, t);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cout) base[(size_t)Eng::out_index(a.plan, t, m) * stride] = v[m];
    }
}

// ---------------------------------------------------------------------------
// fused z pass: forward z FFT -> k-space operator(s) -> inverse z FFT
// ---------------------------------------------------------------------------
enum { ZM_GRAD = 0, ZM_DIV = 1, ZM_ABS = 2 };

struct ZArgs {
    int zero;                // always 0 (see the salt in kw_xvel)
    const float2 *in[3];
    float2 *out[3];
    GridDev g;
    Tables t;
    FftPlan pf, pi;          // forward plan and the plan of the inverse
    int tb;
    int ntiles;              // column tiles per ky row
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
        const float s = kappa_of_x2(a.g.half_cdt * a.g.half_cdt * k2) * a.g.inv_n;
        float2 d;
        if (MODE == ZM_GRAD)
            d = (o == 0) ? a.t.dpx[ix] : (o == 1) ? a.t.dpy[iy] : a.t.dpz[iz];
        else
            d = (o == 0) ? a.t.dmx[ix] : (o == 1) ? a.t.dmy[iy] : a.t.dmz[iz];
        return c_scale(d, s);
    }
}

// kw_zfused: a block handles a tile of tb columns of one ky row (column 0 is
// skipped on store); kw_zpair handles column 0: it holds X0 + i XN
// (kx = 0 part and Nyquist part, both real before the y/z transforms).  After
// the forward z transform the parts are separated with the conjugate-symmetric
// partner at (-ky, -kz):
//   A = (C(ky,kz) + conj C(-ky,-kz)) / 2,   B = (C(ky,kz) - conj C(-ky,-kz)) / 2i
// each gets its own operator and the results are repacked as A' + i B'.  A pair
// block holds tb/2 pairs of rows (ky, -ky) in adjacent columns of its tile.
template <class Eng, int MODE>
__global__ void __launch_bounds__(512) kw_zfused(ZArgs a) {
    constexpr int E = Eng::E;
    extern __shared__ float2 sh[];
    const int tid = threadIdx.x;
    const int b = tid % a.tb, t = tid / a.tb;
    const int ny = a.g.ny, M = a.g.M;
    const size_t stride = (size_t)M * ny;
    const ColLds lds{sh, a.tb, b};
    const int blk = blockIdx.x;
    const int cin = Eng::in_count(a.pf, t);
    const int cmid = Eng::out_count(a.pf, t);
    const int cout = Eng::out_count(a.pi, t);
    // blockIdx.y selects the output; each output has its own blocks (the
    // gradient's three outputs re-read the one input), which keeps a block to
    // one forward and one inverse transform and its register use low
    const int o = blockIdx.y;
    const int f = (MODE == ZM_GRAD) ? 0 : o;

    const int tile = blk % a.ntiles, iy = blk / a.ntiles;
    const int col = tile * a.tb + b;
    const bool ok = col < M;
    const bool st_ok = ok && col != 0;
    const int ix = ok ? col : 0;
    const size_t off = (size_t)iy * M + col;
    float2 v[E];
    if (ok) {
        const float2 *src = pick3(a.in, f) + off;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = src[(size_t)Eng::in_index(a.pf, t, m) * stride];
    }
    Eng::template run<false>(a.pf, a.t.tw_z, t, lds, v);
#pragma unroll
    for (int m = 0; m < E; ++m)
        if (m < cmid) v[m] = c_mul(v[m], z_operator<MODE>(a, o, ix, iy, Eng::out_index(a.pf, t, m)));
    Eng::template run<true>(a.pi, a.t.tw_z, t, lds, v);
    if (st_ok) {
        float2 *dst = pick3(a.out, o) + off;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cout) dst[(size_t)Eng::out_index(a.pi, t, m) * stride] = v[m];
    }
}

template <class Eng, int MODE>
__global__ void __launch_bounds__(512) kw_zpair(ZArgs a) {
    constexpr int E = Eng::E;
    extern __shared__ float2 sh[];
    const int tid = threadIdx.x;
    const int b = tid % a.tb, t = tid / a.tb;
    const int ny = a.g.ny, nz = a.g.nz, M = a.g.M;
    const size_t stride = (size_t)M * ny;
    // LDS: [FFT exchange buffer | forward spectra of the block's columns]
    const ColLds lds{sh, a.tb, b};
    const ColLds spec{sh + (size_t)a.tb * nz, a.tb, b};
    const ColLds partner{sh + (size_t)a.tb * nz, a.tb, b ^ 1};
    const int cin = Eng::in_count(a.pf, t);
    const int cmid = Eng::out_count(a.pf, t);
    const int cout = Eng::out_count(a.pi, t);
    const int side = b & 1;
    const int pair = blockIdx.x * (a.tb / 2) + (b >> 1);
    const bool valid = (b < (a.tb & ~1)) && pair <= ny / 2;
    const int ky0 = valid ? pair : 0;
    const int ky1 = (ny - ky0) % ny;
    const int iy = side ? ky1 : ky0;
    const bool store = valid && (side == 0 || ky1 != ky0);
    const size_t off = (size_t)iy * M;
    const int o = blockIdx.y;                       // output (see kw_zfused)
    const int f = (MODE == ZM_GRAD) ? 0 : o;
    float2 v[E];
    if (valid) {
        const float2 *src = pick3(a.in, f) + off;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = src[(size_t)Eng::in_index(a.pf, t, m) * stride];
    }
    Eng::template run<false>(a.pf, a.t.tw_z, t, lds, v);
#pragma unroll
    for (int m = 0; m < E; ++m)
        if (m < cmid) spec.st(Eng::out_index(a.pf, t, m), v[m]);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (m < cmid) {
            const int iz = Eng::out_index(a.pf, t, m);
            const float2 c = v[m];
            const float2 pc = c_conj(partner.ld((nz - iz) % nz));
            const float2 va = c_scale(c_add(c, pc), 0.5f);
            const float2 d = c_sub(c, pc);
            const float2 vb = make_float2(0.5f * d.y, -0.5f * d.x);   // (c - pc) / (2i)
            const float2 ya = c_mul(va, z_operator<MODE>(a, o, 0, iy, iz));
            const float2 yb = c_mul(vb, z_operator<MODE>(a, o, M, iy, iz));
            v[m] = make_float2(ya.x - yb.y, ya.y + yb.x);   // ya + i yb
        }
    }
    Eng::template run<true>(a.pi, a.t.tw_z, t, lds, v);
    if (store) {
        float2 *dst = pick3(a.out, o) + off;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cout) dst[(size_t)Eng::out_index(a.pi, t, m) * stride] = v[m];
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
    FftPlan pf, pi;          // forward plan (length M) and the plan of the inverse
    int tb;                  // rows per block
    const float2 *Sin[3];
    float2 *Sout[3];
    float *fld[3];           // u or rho components
    float *rho_total;
    int zero;                // always 0; mixed into per-iteration addresses (see salt)
    const float *rsrc;       // xfwd: real input
    float *rdst;             // xinv: real output
    float scale;
};

// c2r: packed spectrum row -> v[m] = x[2n] + i x[2n+1], n = out_index(pi, t, m)
// (unnormalised; the result is nx times the inverse DFT)
template <class Eng>
__device__ __forceinline__ void row_c2r(const XArgs &a, const float2 *__restrict__ row, bool ok,
                                        int t, const RowLds &lds, float2 (&v)[Eng::E],
                                        int salt = 0) {
    constexpr int E = Eng::E;
    const int M = a.g.M;
    const float2 *tw_post = a.t.tw_post + salt;
    const int cin = Eng::in_count(a.pi, t);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cin) {
                const int k = Eng::in_index(a.pi, t, m);
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
                const float2 B = c_mulc(D, tw_post[k]);                         // * w^-k
                v[m] = make_float2(A.x - B.y, A.y + B.x);                       // A + i B
            }
        }
    }
    Eng::template run<true>(a.pi, a.t.tw_x + salt, t, lds, v);
}

// r2c: v[m] = x[2n] + i x[2n+1], n = in_index(pf, t, m)  ->  packed spectrum row
template <class Eng>
__device__ __forceinline__ void row_r2c(const XArgs &a, float2 *__restrict__ row, bool ok, int t,
                                        const RowLds &lds, float2 (&v)[Eng::E], int salt = 0) {
    constexpr int E = Eng::E;
    const int M = a.g.M;
    const float2 *tw_post = a.t.tw_post + salt;
    Eng::template run<false>(a.pf, a.t.tw_x + salt, t, lds, v);
    const int cout = Eng::out_count(a.pf, t);
#pragma unroll
    for (int m = 0; m < E; ++m)
        if (m < cout) lds.st(Eng::out_index(a.pf, t, m), v[m]);
    __syncthreads();
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cout) {
                const int k = Eng::out_index(a.pf, t, m);
                const float2 Z = v[m];
                float2 out;
                if (k == 0) {
                    out = make_float2(Z.x + Z.y, Z.x - Z.y);     // X0 + i XN
                } else {
                    const float2 Zm = c_conj(lds.ld(M - k));
                    const float2 A = c_scale(c_add(Z, Zm), 0.5f);
                    const float2 Bh = c_scale(c_sub(Z, Zm), 0.5f);
                    const float2 c = c_mul(tw_post[k], Bh);
                    out = make_float2(A.x + c.y, A.y - c.x);     // A - i w^k B
                }
                row[k] = out;
            }
        }
    }
    __syncthreads();
}

#define KW_XPROLOGUE                                                   \
    constexpr int E = Eng::E;                                          \
    extern __shared__ float2 sh[];                                     \
    const int L = a.pf.L;                                              \
    const int tid = threadIdx.x, t = tid % L, b = tid / L;             \
    const int row = blockIdx.x * a.tb + b;                             \
    const bool ok = row < a.g.rows;                                    \
    const int rr = ok ? row : 0;                                       \
    const int M = a.g.M, nx = a.g.nx;                                  \
    const RowLds lds{sh, b * row_pitch(M)};                            \
    const size_t rbase = (size_t)rr * nx;                              \
    const int cupd = Eng::out_count(a.pi, t);                          \
    (void)nx; (void)rbase; (void)cupd;

// The three velocity components are independent: blockIdx.y selects one.
template <class Eng>
__global__ void __launch_bounds__(512) kw_xvel(XArgs a) {
    KW_XPROLOGUE
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const int xi = blockIdx.y;
    float2 v[E];
    row_c2r<Eng>(a, pick3(a.Sin, xi) + (size_t)rr * M, ok, t, lds, v);
    if (ok) {
        float *u = pick3(a.fld, xi);
        const Coef dtr = xi == 0 ? a.m.dtr[0] : xi == 1 ? a.m.dtr[1] : a.m.dtr[2];
        const float qy = a.t.pml_sy[iy], qz = a.t.pml_sz[iz];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const int x = 2 * Eng::out_index(a.pi, t, m);
                const size_t i = rbase + x;
                float2 q;
                if (xi == 0) q = make_float2(a.t.pml_sx[x], a.t.pml_sx[x + 1]);
                else if (xi == 1) q = make_float2(qy, qy);
                else q = make_float2(qz, qz);
                const float2 d = coef2_at(dtr, i);
                const float2 u0 = ld2(u, i);
                const float2 g = v[m];
                float2 un;
                un.x = q.x * (q.x * u0.x - d.x * g.x);
                un.y = q.y * (q.y * u0.y - d.y * g.y);
                st2(u, i, un);
                v[m] = un;
            }
        }
    }
    row_r2c<Eng>(a, pick3(a.Sout, xi) + (size_t)rr * M, ok, t, lds, v);
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
template <class Eng>
__device__ __forceinline__ void record_mask(const XArgs &a, float *line, int row, bool ok, int t,
                                            int L, int b, int step, const float2 (&p)[Eng::E]) {
    constexpr int E = Eng::E;
    const int nx = a.g.nx;
    int beg = 0, end = 0;
    if (ok) {
        beg = a.sen.row_ptr[row];
        end = a.sen.row_ptr[row + 1];
    }
    const bool any = __syncthreads_or(end > beg);
    if (!any) return;
    float *mine = line + (size_t)b * nx;
    const int cnt = Eng::out_count(a.pi, t);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cnt) {
                const int x = 2 * Eng::out_index(a.pi, t, m);
                mine[x] = p[m].x;
                mine[x + 1] = p[m].y;
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

// sensors, non-finite check and x r2c of the new pressure (v holds p in the
// output layout of the inverse x transform)
template <class Eng>
__device__ __forceinline__ void finish_pressure(const XArgs &a, float *line, int row, bool ok,
                                                int t, int L, int b, const RowLds &lds,
                                                float2 (&v)[Eng::E]) {
    constexpr int E = Eng::E;
    const int M = a.g.M, nx = a.g.nx;
    const size_t rbase = (size_t)(ok ? row : 0) * nx;
    const int step = *a.cnt.step;
    const bool rec = step >= a.sen.record_start;
    const int cnt = Eng::out_count(a.pi, t);
    bool bad = false;
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cnt) {
                const float2 p = v[m];
                bad |= !(__builtin_isfinite(p.x) && __builtin_isfinite(p.y));
                if (rec && a.sen.all_points) {
                    const size_t i = rbase + 2 * Eng::out_index(a.pi, t, m);
                    if (a.sen.p_max) {
                        const float2 mx = ld2(a.sen.p_max, i);
                        st2(a.sen.p_max, i, make_float2(fmaxf(mx.x, p.x), fmaxf(mx.y, p.y)));
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
        record_mask<Eng>(a, line, row, ok, t, L, b, step, v);
    row_r2c<Eng>(a, a.Sout[0] + (size_t)(ok ? row : 0) * M, ok, t, lds, v);
}

template <class Eng>
__global__ void __launch_bounds__(512) kw_xden(XArgs a) {
    KW_XPROLOGUE
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    float *line = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M));
    const float dt = a.g.dt;
    const bool has_src = scatter_source(a, line, rr, ok, t, L, b);
    const float *mysrc = line + (size_t)b * nx;

    float2 acc_rho[E], acc_div[E];
#pragma unroll
    for (int m = 0; m < E; ++m) acc_rho[m] = acc_div[m] = make_float2(0.0f, 0.0f);

#pragma unroll 1
    for (int xi = 0; xi < 3; ++xi) {
        const int salt = xi & a.zero;      // see kw_xvel
        float2 v[E];
        row_c2r<Eng>(a, pick3(a.Sin, xi) + (size_t)rr * M, ok, t, lds, v, salt);
        if (ok) {
            float *rho = pick3(a.fld, xi);
            const float qy = a.t.pml_y[iy], qz = a.t.pml_z[iz];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cupd) {
                    const int x = 2 * Eng::out_index(a.pi, t, m);
                    const size_t i = rbase + x;
                    float2 q;
                    if (xi == 0) q = make_float2(a.t.pml_x[x + salt], a.t.pml_x[x + 1 + salt]);
                    else if (xi == 1) q = make_float2(qy, qy);
                    else q = make_float2(qz, qz);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    const float2 d = v[m];
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
                    acc_rho[m] = c_add(acc_rho[m], nw);
                    acc_div[m] = c_add(acc_div[m], d);
                }
            }
        }
    }

    float2 v[E];
    if (a.m.absorbing) {
        // store rho = sum rho_xi for the equation of state, transform rho0 sum du and rho
        if (ok) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cupd) {
                    const size_t i = rbase + 2 * Eng::out_index(a.pi, t, m);
                    st2(a.rho_total, i, acc_rho[m]);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    v[m] = make_float2(r0.x * acc_div[m].x, r0.y * acc_div[m].y);
                }
            }
        }
        row_r2c<Eng>(a, a.Sout[0] + (size_t)rr * M, ok, t, lds, v);
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = acc_rho[m];
        row_r2c<Eng>(a, a.Sout[1] + (size_t)rr * M, ok, t, lds, v);
    } else {
        if (ok) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cupd) {
                    const size_t i = rbase + 2 * Eng::out_index(a.pi, t, m);
                    const float2 rho = acc_rho[m];
                    const float2 c2 = coef2_at(a.m.c0sq, i);
                    float2 p = make_float2(c2.x * rho.x, c2.y * rho.y);
                    if (a.m.nonlinear) {
                        const float2 nl = coef2_at(a.m.nl, i);
                        p.x += nl.x * rho.x * rho.x;
                        p.y += nl.y * rho.y * rho.y;
                    }
                    v[m] = p;
                }
            }
        }
        finish_pressure<Eng>(a, line, rr, ok, t, L, b, lds, v);
    }
}

template <class Eng>
__global__ void __launch_bounds__(512) kw_xeos(XArgs a) {
    KW_XPROLOGUE
    float *line = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M));
    float2 va[E], v[E];
    row_c2r<Eng>(a, a.Sin[0] + (size_t)rr * M, ok, t, lds, va);
    row_c2r<Eng>(a, a.Sin[1] + (size_t)rr * M, ok, t, lds, v);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const size_t i = rbase + 2 * Eng::out_index(a.pi, t, m);
                const float2 rho = ld2(a.rho_total, i);
                const float2 c2 = coef2_at(a.m.c0sq, i);
                const float2 ta = coef2_at(a.m.ta, i);
                const float2 tb = coef2_at(a.m.tb, i);
                float2 p;
                p.x = c2.x * rho.x + ta.x * va[m].x + tb.x * v[m].x;
                p.y = c2.y * rho.y + ta.y * va[m].y + tb.y * v[m].y;
                if (a.m.nonlinear) {
                    const float2 nl = coef2_at(a.m.nl, i);
                    p.x += nl.x * rho.x * rho.x;
                    p.y += nl.y * rho.y * rho.y;
                }
                v[m] = p;
            }
        }
    }
    finish_pressure<Eng>(a, line, rr, ok, t, L, b, lds, v);
}

template <class Eng>
__global__ void __launch_bounds__(512) kw_xfwd(XArgs a) {
    KW_XPROLOGUE
    float2 v[E];
    const int cin = Eng::in_count(a.pf, t);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = ld2(a.rsrc, rbase + 2 * Eng::in_index(a.pf, t, m));
    }
    row_r2c<Eng>(a, a.Sout[0] + (size_t)rr * M, ok, t, lds, v);
}

template <class Eng>
__global__ void __launch_bounds__(512) kw_xinv(XArgs a) {
    KW_XPROLOGUE
    float2 v[E];
    row_c2r<Eng>(a, a.Sin[0] + (size_t)rr * M, ok, t, lds, v);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cupd) st2(a.rdst, rbase + 2 * Eng::out_index(a.pi, t, m), c_scale(v[m], a.scale));
    }
}

// engine dispatch ---------------------------------------------------------------
#define KW_ENGINE_SWITCH(ENG, BODY)                                            \
    switch (ENG) {                                                             \
    case ENG_G16: { using Eng = EngGeneric<16>; BODY; } break;                 \
    case ENG_G32: { using Eng = EngGeneric<32>; BODY; } break;                 \
    case ENG_F8:  { using Eng = EngFixed<8>; BODY; } break;                    \
    default:      { using Eng = EngFixed<16>; BODY; } break;                   \
    }

}  // namespace kw
