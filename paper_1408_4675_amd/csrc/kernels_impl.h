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
// along (the y pass stores it unpacked between its forward and inverse
// transforms, see col0_type), and the fused z pass applies to each part the
// operator of its own kx (0 or Nyquist).
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
// Element at a 32-bit byte offset from p, p uniform over the wavefront (a
// requirement: the first active lane's p is used for all).  p
// is read into scalar registers (readfirstlane) and accessed as global memory,
// so that each access is one instruction with a scalar base and a vector
// offset: no 64-bit address arithmetic per element (left to itself the
// compiler re-associates base and offset into 64-bit vector multiply-adds).
// The column passes keep their per-lane offsets below 4 GiB (checked when a
// simulation is set up).
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ gchar *global_uniform(const void *p) {
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<gchar *>(((uint64_t)hi << 32) | lo);
}
typedef float vf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_at(const float2 *p, uint32_t off) {
    const vf2 x = *reinterpret_cast<const __attribute__((address_space(1))) vf2 *>(global_uniform(p) + off);
    return make_float2(x.x, x.y);
}
__device__ __forceinline__ void st_at(float2 *p, uint32_t off, float2 v) {
    vf2 x;
    x.x = v.x;
    x.y = v.y;
    *reinterpret_cast<__attribute__((address_space(1))) vf2 *>(global_uniform(p) + off) = x;
}
// A pair of real grid values (x, x + 1) of a row of an x-pass block: element
// index u, uniform over the block, plus a per-lane byte offset l (row within
// the block and x), so that one lane offset serves every field and element
// of a thread.
struct XPos {
    size_t u;
    uint32_t l;
};
__device__ __forceinline__ float2 ld2(const float *p, XPos e) {
    return ld_at(reinterpret_cast<const float2 *>(p + e.u), e.l);
}
__device__ __forceinline__ void st2(float *p, XPos e, float2 v) {
    st_at(reinterpret_cast<float2 *>(p + e.u), e.l, v);
}
__device__ __forceinline__ float2 coef2_at(const Coef &c, XPos e) {
    if (c.map) return ld2(c.map, e);
    return make_float2(c.scalar, c.scalar);
}

// select one of three values without indexing the argument array at run time
// (a run-time index into a by-value kernel argument forces it into scratch)
template <class T>
__device__ __forceinline__ T pick3v(T p0, T p1, T p2, int i) {
    return i == 0 ? p0 : (i == 1 ? p1 : p2);
}
#define pick3(arr, i) pick3v((arr)[0], (arr)[1], (arr)[2], (i))

// sin(x)/x for x = sqrt(x2) beyond the polynomial's range (time steps far above
// the usual CFL numbers); kept out of line so that the unrolled operator loops
// of the z passes carry one call instead of sixteen copies of sinf
__device__ __attribute__((noinline)) float kappa_large(float x2) {
    const float x = sqrtf(x2);
    return sinf(x) / x;
}

// kappa = sinc(x) = sin(x)/x with x^2 = (c_ref dt / 2)^2 k^2, evaluated as its
// Taylor polynomial in x^2 up to x^16/17! (truncation error below 1e-9 for
// x <= 1.7, which covers CFL numbers up to about 0.6 at the corner of the
// wavenumber cube); larger arguments take kappa_large.  No sqrt and no range
// reduction on the common path.
__device__ __forceinline__ float kappa_of_x2(float x2) {
    if (x2 > 2.89f) return kappa_large(x2);
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
// Column kx = 0 of a spectrum holds X0 + i XN (the kx = 0 and Nyquist parts of
// the x transform, both real functions of (y, z)).  Their y transforms A(ky),
// B(ky) are Hermitian in ky, so between the forward and the inverse y pass
// column 0 is stored unpacked, with h = (ny - 1) / 2:
//   row 0 (and row ny/2 for even ny): A + i B as computed (there A and B are
//                                      real functions of z);
//   rows 1..h:                         A(ky = row);
//   rows ny-h..ny-1:                   B(ky = row - (ny - 1 - h)).
// The fused z pass then treats these rows as ordinary columns (kx = 0 for A,
// the Nyquist kx for B) and separates A and B of rows 0 and ny/2 with the
// kz <-> -kz partner in the same column.
// ---------------------------------------------------------------------------
enum { C0_DOUBLE = 0, C0_A = 1, C0_B = 2 };
__device__ __forceinline__ int col0_type(int r, int ny) {
    const int h = (ny - 1) / 2;
    if (r == 0 || (!(ny & 1) && r == ny / 2)) return C0_DOUBLE;
    return r <= h ? C0_A : C0_B;
}
// ky index of row r of the unpacked column 0
__device__ __forceinline__ int col0_ky(int r, int ny) {
    const int h = (ny - 1) / 2;
    if (r == 0 || r <= h || (!(ny & 1) && r == ny / 2)) return r;
    return r - (ny - 1 - h);
}

// Twiddle tables are read from LDS inside the transforms: every kernel copies
// the ones it needs to the start of its dynamic LDS first (a global read per
// twiddle inside each pass put a memory latency on every pass).
__device__ __forceinline__ void stage_table(float2 *dst, const float2 *__restrict__ src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// XCD-aware order of the column passes.  Workgroups are dispatched round-robin
// over the 8 XCDs (XCD = workgroup id mod 8), each with an L2 of its own.
// Blocks that read the same 128-byte lines -- G consecutive tiles narrower than
// a line, and R blocks of one tile that each read its input -- are given
// consecutive dispatch slots on one XCD, so that all but the first find the
// lines in that XCD's L2 instead of fetching them again.  Workgroup B maps to
// tile block `blk` and repeat `r`; false for the padding of the grid (whole
// groups on every XCD).
__host__ __device__ inline int xcd_grid(int nblk, int G, int R) {
    const int groups = (nblk + G - 1) / G;
    return (groups + 7) / 8 * 8 * G * R;
}
__device__ __forceinline__ bool xcd_order(int B, int G, int R, int nblk, int &blk, int &r) {
    const int x = B & 7, q = B >> 3, GR = G * R;
    const int w = q % GR;
    blk = ((q / GR) * 8 + x) * G + w / R;
    r = w % R;
    return blk < nblk;
}
// tiles sharing a 128-byte line: G = 16 / tb for tiles under 16 columns
__host__ __device__ inline int line_group(int tb) { return tb < 16 ? 16 / tb : 1; }

// Drive value s_e of element e in step n, at t = (n + t_offset) dt (n + 1/2
// for the mass source of Eq. (4d), n for the force of Eq. (4b), n + 1 for a
// pressure source): a_e sin(omega t + phi_e) = a_e cos(phi_e) sin(omega t)
// + a_e sin(phi_e) cos(omega t) in float64, or the sampled signal.
__device__ __forceinline__ float drive_at(const SourceDev &src, int e, int n) {
    if (src.signal) return (n < src.n_samples) ? src.signal[(size_t)e * src.n_samples + n] : 0.0f;
    const double th = src.omega_dt * ((double)n + src.t_offset);
    return (float)(src.amp_cos[e] * sin(th) + src.amp_sin[e] * cos(th));
}

// ---------------------------------------------------------------------------
// y pass: in-place column FFTs of up to three spectra
// ---------------------------------------------------------------------------
struct YArgs {
    float2 *f[3];
    float2 *o[3];            // destinations (the same as f for an in-place pass)
    int M, ny;
    FftPlan plan;            // forward plan, or the reversed plan for the inverse
    const float2 *tw;
    int tb;
    int ntiles, nz;          // column tiles per y-z plane row, z planes
    // prologue (first kernel of a step): advance the step counter and
    // evaluate the drive value of every source element at t = (n + 1/2) dt
    int prologue;
    Counters cnt;
    SourceDev src;
    // and cos, sin of h w t (h = 1..n_harm) at t = (n + 1) dt, the time of
    // the pressure this step produces, for the harmonic sums of the sensors
    float *hw;
    int n_harm;
    double harm_wdt;
};

// MAXT: 512, or 1024 for the wide column tiles of long axes (fixed engines
// only, whose register count fits the 128 registers a 1024-thread block allows)
template <class Eng, bool INV, int MAXT = 512>
__global__ void __launch_bounds__(MAXT) kw_ypass(YArgs a) {
    constexpr int E = Eng::E;
    extern __shared__ float2 lds_all[];
    float2 *const tws = lds_all;             // ny twiddles
    float2 *const sh = lds_all + a.ny;       // column tile
    const int tid = threadIdx.x;
    const int b = tid % a.tb, t = tid / a.tb;
    int blk, rep_;
    if (!xcd_order(blockIdx.x, line_group(a.tb), 1, a.ntiles * a.nz, blk, rep_)) return;
    const int tile = blk % a.ntiles, iz = blk / a.ntiles;
    const int col = tile * a.tb + b;
    const bool ok = col < a.M;
    // element (row t + m step, column col) of this block's tile: uniform base
    // base + m step M, lane offset (t M + b) elements
    const size_t tile_off = (size_t)iz * a.ny * a.M + (size_t)tile * a.tb;
    const float2 *const base = pick3(a.f, (int)blockIdx.z) + tile_off;
    const uint32_t lane = (uint32_t)(t * a.M + b) * 8u;

    if constexpr (!INV) {
        // (a call to an out-of-line prologue costs the kernel a stack frame:
        // scratch memory and more registers for every block)
        if (a.prologue && blk == 0 && blockIdx.z == 0) {
            const int n = *a.cnt.step;
            __syncthreads();
            if (tid == 0) *a.cnt.step = n + 1;
            for (int e = tid; e < a.src.n_elements; e += blockDim.x) a.src.drive[e] = drive_at(a.src, e, n);
            for (int h = tid; h < a.n_harm; h += blockDim.x) {
                const double th = a.harm_wdt * (double)(h + 1) * (double)(n + 1);
                a.hw[2 * h] = (float)cos(th);
                a.hw[2 * h + 1] = (float)sin(th);
            }
        }
    }

    float2 v[E];
    const int ny = a.ny, h = (ny - 1) / 2;
    const ColLds lds{sh, a.tb, b};
    const int cin = Eng::in_count(a.plan, t);
    if (ok) {
        const size_t jump = (size_t)Eng::in_step(a.plan) * a.M;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = ld_at(base + m * jump, lane);
    }
    stage_table(tws, a.tw, ny);
    __syncthreads();
    const bool tile0 = tile == 0;                // block-uniform
    if (INV && tile0) {
        // repack column 0: C(ky) = A(ky) + i B(ky), using A(-ky) = conj A(ky)
        if (b == 0) {
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cin) lds.st(Eng::in_index(a.plan, t, m), v[m]);
        }
        __syncthreads();
        if (b == 0) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cin) {
                    const int ky = Eng::in_index(a.plan, t, m);
                    if (col0_type(ky, ny) != C0_DOUBLE) {
                        const bool neg = ky > h;                 // ky = ny - j, j = 1..h
                        const int j = neg ? ny - ky : ky;
                        float2 A = lds.ld(j), B = lds.ld(ny - 1 - h + j);
                        if (neg) {
                            A = c_conj(A);
                            B = c_conj(B);
                        }
                        v[m] = make_float2(A.x - B.y, A.y + B.x);   // A + i B
                    }
                }
            }
        }
        __syncthreads();
    }
    Eng::template run<INV>(a.plan, tws, t, lds, v);
    const int cout = Eng::out_count(a.plan, t);
    if (!INV && tile0) {
        // unpack column 0 into A (rows 1..h) and B (rows ny-h..ny-1)
        if (b == 0) {
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cout) lds.st(Eng::out_index(a.plan, t, m), v[m]);
        }
        __syncthreads();
        if (b == 0) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cout) {
                    const int r = Eng::out_index(a.plan, t, m);
                    const int type = col0_type(r, ny);
                    if (type != C0_DOUBLE) {
                        const int j = col0_ky(r, ny);
                        const float2 c = lds.ld(j);
                        const float2 pc = c_conj(lds.ld(ny - j));
                        if (type == C0_A) {
                            v[m] = c_scale(c_add(c, pc), 0.5f);                 // (C + conj C(-ky)) / 2
                        } else {
                            const float2 d = c_sub(c, pc);
                            v[m] = make_float2(0.5f * d.y, -0.5f * d.x);        // (C - conj C(-ky)) / 2i
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (ok) {
        float2 *const obase = pick3(a.o, (int)blockIdx.z) + tile_off;
        const size_t jump = (size_t)Eng::out_step(a.plan) * a.M;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cout) st_at(obase + m * jump, lane, v[m]);
    }
}

// ---------------------------------------------------------------------------
// fused z pass: forward z FFT -> k-space operator(s) -> inverse z FFT
// ---------------------------------------------------------------------------
// (z-pass modes ZM_* are defined in kw_internal.h)

struct ZArgs {
    int zero;                // always 0 (see the salt of the gradient in kw_zfused)
    const float2 *in[3];
    const float2 *add0[2];   // ABS, ABSM: addends of input 0 (summed as it is loaded), or null
    float2 *out[3];
    GridDev g;
    Tables t;
    FftPlan pf, pi;          // forward plan and the plan of the inverse
    int tb;
    int ntiles;              // column tiles per ky row
    float sa, sb;            // ABSM: c0^2 tau and -c0^2 eta of a homogeneous medium
                             // (times a factor of input 0's scaling); ABS: sa scales input 0
};

// kz of FFT index iz (Eq. (5)): m 2 pi / (nz dz), m = iz - nz above the middle
__device__ __forceinline__ float kz_of(const GridDev &g, int iz) {
    return (float)(iz <= (g.nz - 1) / 2 ? iz : iz - g.nz) * g.dkz;
}

// multiplier of output o at (kx index ix (M = Nyquist), ky index iy, kz index iz)
// dzl: the z factor D+-_z of the mode, staged in LDS
template <int MODE>
__device__ __forceinline__ float2 z_operator(const ZArgs &a, int o, int ix, int iy, int iz,
                                             const float2 *dzl) {
    const float kx = a.t.kx[ix], ky = a.t.ky[iy], kz = kz_of(a.g, iz);
    const float k2 = kx * kx + ky * ky + kz * kz;
    if constexpr (MODE == ZM_ABS) {
        if (k2 <= 0.0f) return make_float2(0.0f, 0.0f);
        const float e = (o == 0) ? a.g.y_tau : a.g.y_eta;
        // k^(y-2), k^(y-1) = 2^(e log2 k^2) with the hardware log2 and exp2
        // (about 1 ulp each): k^2 > 0 and the powers are normal floats for
        // any grid spacing in use, so the library's denormal and range
        // handling (a tenth of this pass's vector instructions) is not needed
        return make_float2(__builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(k2)) * a.g.inv_n, 0.0f);
    } else {
        const float s = kappa_of_x2(a.g.half_cdt * a.g.half_cdt * k2) * a.g.inv_n;
        float2 d;
        if (MODE == ZM_GRAD || MODE == ZM_GRADT)
            d = (o == 0) ? a.t.dpx[ix] : (o == 1) ? a.t.dpy[iy] : dzl[iz];
        else
            d = (o == 0) ? a.t.dmx[ix] : (o == 1) ? a.t.dmy[iy] : dzl[iz];
        if constexpr (MODE == ZM_DIVT || MODE == ZM_GRADT) d = c_conj(d);
        return c_scale(d, s);
    }
}

// kw_zfused: a block handles a tile of tb columns of one ky row, for one
// output (blockIdx.y).  Column 0 arrives unpacked by the y pass: an A row takes
// the operator of kx = 0 at its own ky, a B row the operator of the Nyquist kx.
// Rows 0 and ny/2 still hold A + i B with A, B real in z; after the forward z
// transform the two parts are separated with the partner at -kz,
//   A = (C(kz) + conj C(-kz)) / 2,   B = (C(kz) - conj C(-kz)) / 2i,
// each gets its own operator, and the results are repacked as A' + i B'.
// Per-block context of the fused z pass (one tile of columns of one ky row).
struct ZCtx {
    int t, b, iy, ix, iyk, M;
    bool ok, pairing;
    size_t off;              // element offset of the tile (uniform): iy M + first column
    size_t stride;           // element distance of consecutive z
    uint32_t lane;           // byte offset of (z = t, column b) from the tile
    ColLds lds;
    const float2 *tws;
    const float2 *dzl;
};

template <class Eng>
__device__ __forceinline__ void z_load(const ZArgs &a, const ZCtx &c, const float2 *src,
                                       float2 (&v)[Eng::E]) {
    constexpr int E = Eng::E;
    const int cin = Eng::in_count(a.pf, c.t);
    if (c.ok) {
        const float2 *const base = src + c.off;
        const size_t jump = (size_t)Eng::in_step(a.pf) * c.stride;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = ld_at(base + m * jump, c.lane);
    }
}

// store of the inverse transform's output layout
template <class Eng>
__device__ __forceinline__ void z_store(const ZArgs &a, const ZCtx &c, float2 *dst,
                                        const float2 (&v)[Eng::E]) {
    constexpr int E = Eng::E;
    const int cout = Eng::out_count(a.pi, c.t);
    if (c.ok) {
        float2 *const base = dst + c.off;
        const size_t jump = (size_t)Eng::out_step(a.pi) * c.stride;
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cout) st_at(base + m * jump, c.lane, v[m]);
    }
}

// v (a forward z spectrum) times the operator `o` of OPMODE times `scale`
template <class Eng, int OPMODE>
__device__ __forceinline__ void z_op(const ZArgs &a, const ZCtx &c, int o, float scale,
                                     float2 (&v)[Eng::E]) {
    constexpr int E = Eng::E;
    const int t = c.t, b = c.b, iy = c.iy, M = c.M;
    const ColLds &lds = c.lds;
    const int cmid = Eng::out_count(a.pf, t);
    if (c.pairing && b == 0) {
        // the raw spectrum of the double row goes to LDS column 0 (free after
        // the transform's trailing barrier) for the pair loop below
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cmid) lds.st(Eng::out_index(a.pf, t, m), v[m]);
    }
#pragma unroll
    for (int m = 0; m < E; ++m)
        if (m < cmid)
            v[m] = c_mul(v[m], c_scale(z_operator<OPMODE>(a, o, c.ix, c.iyk, Eng::out_index(a.pf, t, m),
                                                          c.dzl), scale));
    if (c.pairing) {
        // (kz, -kz) pairs of the double row, one pair per iteration and thread,
        // updated in place in LDS (a pair is read and written by one thread)
        __syncthreads();
        if (b == 0) {
            const int nz = a.g.nz, nth = blockDim.x / a.tb;
            for (int iz = t; iz <= nz / 2; iz += nth) {
                const int jz = (nz - iz) % nz;
                const float2 c1 = lds.ld(iz), c2 = lds.ld(jz);
                // A(kz) = (C(kz) + conj C(-kz)) / 2, B(kz) = (C(kz) - conj C(-kz)) / 2i
                const float2 s1 = c_add(c1, c_conj(c2)), d1 = c_sub(c1, c_conj(c2));
                const float2 A1 = c_scale(s1, 0.5f * scale);
                const float2 B1 = make_float2(0.5f * scale * d1.y, -0.5f * scale * d1.x);
                const float2 ya = c_mul(A1, z_operator<OPMODE>(a, o, 0, iy, iz, c.dzl));
                const float2 yb = c_mul(B1, z_operator<OPMODE>(a, o, M, iy, iz, c.dzl));
                lds.st(iz, make_float2(ya.x - yb.y, ya.y + yb.x));          // ya + i yb
                if (jz != iz) {
                    // A(-kz) = conj A(kz), B(-kz) = conj B(kz)
                    const float2 za = c_mul(c_conj(A1), z_operator<OPMODE>(a, o, 0, iy, jz, c.dzl));
                    const float2 zb = c_mul(c_conj(B1), z_operator<OPMODE>(a, o, M, iy, jz, c.dzl));
                    lds.st(jz, make_float2(za.x - zb.y, za.y + zb.x));
                }
            }
        }
        __syncthreads();
        if (b == 0) {
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cmid) v[m] = lds.ld(Eng::out_index(a.pf, t, m));
        }
        __syncthreads();
    }
}

// forward z transform of v, then the operator `o` of OPMODE times `scale`
template <class Eng, int OPMODE>
__device__ __forceinline__ void z_fwd_op(const ZArgs &a, const ZCtx &c, int o, float scale,
                                         float2 (&v)[Eng::E]) {
    Eng::template run<false>(a.pf, c.tws, c.t, c.lds, v);
    z_op<Eng, OPMODE>(a, c, o, scale, v);
}

// SPLIT (gradient only): one block per output, as for the generic engines,
// instead of one block that keeps the forward spectrum for all three (the
// kept spectrum holds 32 more registers, too many for two 512-thread blocks
// per CU on long columns)
template <class Eng, int MODE, int MAXT = 512, bool SPLIT = false>
__global__ void __launch_bounds__(MAXT) kw_zfused(ZArgs a) {
    constexpr int E = Eng::E;
    // LDS: nz twiddles, nz z factors, then the column tile
    extern __shared__ float2 lds_all[];
    float2 *const tws = lds_all;
    float2 *const dzl = lds_all + a.g.nz;
    float2 *const sh = lds_all + zpass_table_slots(a.g.nz);
    const int tid = threadIdx.x;
    const int b = tid % a.tb, t = tid / a.tb;
    const int ny = a.g.ny, M = a.g.M;
    // The divergence and absorption outputs read inputs of their own: each
    // output has its own blocks (blockIdx.y = output), which keeps a block to
    // one forward and one inverse transform and its register use low.  The
    // gradient's three outputs share one input.  With the fixed engines its
    // block transforms the tile once and runs the three operators and
    // inverse transforms from the kept spectrum (the pass is bound by vector
    // ALU work, and this saves two of the six transforms of a tile).  The
    // generic engines' register arrays are sized for their largest radix and
    // a kept spectrum would cost them two wavefronts per SIMD, so their
    // gradient keeps one block per output (so does a SPLIT instantiation of a
    // fixed engine), and the three blocks of a tile come one after another on
    // one XCD (xcd_order): the second and third reads of the tile hit that
    // XCD's L2.  The merged absorption (ABSM) block transforms both inputs and
    // writes one output.
    constexpr bool fused_grad = MODE == ZM_GRAD && Eng::fixed && Eng::E <= 16 && !SPLIT;
    constexpr int R = (MODE == ZM_GRAD && !fused_grad) ? 3 : 1;
    int blk, o;
    if (!xcd_order(blockIdx.x, line_group(a.tb), R, a.ntiles * a.g.ny, blk, o)) return;
    if constexpr (MODE != ZM_GRAD) o = blockIdx.y;
    const int f = (MODE == ZM_GRAD) ? 0 : o;

    ZCtx c;
    c.t = t;
    c.b = b;
    c.M = M;
    const int tile = blk % a.ntiles;
    c.iy = blk / a.ntiles;
    const int col = tile * a.tb + b;
    c.ok = col < M;
    c.stride = (size_t)M * ny;
    c.off = (size_t)c.iy * M + (size_t)tile * a.tb;
    c.lane = (uint32_t)((size_t)t * c.stride + b) * 8u;
    c.lds = ColLds{sh, a.tb, b};
    c.tws = tws;
    c.dzl = dzl;
    // column 0 of this row (see col0_type): A rows take kx = 0, B rows the
    // Nyquist kx, and the double rows are split with their kz <-> -kz partner
    const int c0type = col0_type(c.iy, ny);
    c.pairing = tile == 0 && c0type == C0_DOUBLE;                  // block-uniform
    c.ix = c.ok ? col : 0;
    c.iyk = c.iy;
    if (col == 0 && c0type != C0_DOUBLE) {
        c.ix = (c0type == C0_A) ? 0 : M;
        c.iyk = col0_ky(c.iy, ny);
    }
    float2 v[E];
    z_load<Eng>(a, c, (MODE == ZM_ABSM) ? a.in[0] : pick3(a.in, f), v);
    if constexpr (MODE == ZM_ABS || MODE == ZM_ABSM) {
        if (f == 0 && a.add0[0]) {                       // block-uniform
            // input 0 is the sum in[0] + add0[0] + add0[1]
            float2 w[E];
            z_load<Eng>(a, c, a.add0[0], w);
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = c_add(v[m], w[m]);
            z_load<Eng>(a, c, a.add0[1], w);
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = c_add(v[m], w[m]);
        }
    }
    stage_table(tws, a.t.tw_z, a.g.nz);
    if constexpr (MODE != ZM_ABS && MODE != ZM_ABSM)
        stage_table(dzl, (MODE == ZM_GRAD || MODE == ZM_GRADT) ? a.t.dpz : a.t.dmz, a.g.nz);
    __syncthreads();
    if constexpr (fused_grad) {
        Eng::template run<false>(a.pf, c.tws, t, c.lds, v);
        float2 S[E];
#pragma unroll
        for (int m = 0; m < E; ++m) S[m] = v[m];
#pragma unroll 1
        for (int oo = 0; oo < 3; ++oo) {
            // salt = 0, unknown to the compiler: the indices of this output are
            // recomputed rather than hoisted out of the loop into registers
            const int salt = oo * a.zero;
            ZCtx cs = c;
            cs.t = t + salt;
            cs.lane = c.lane + salt;
            cs.lds.b = b + salt;
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = S[m];
            z_op<Eng, ZM_GRAD>(a, cs, oo, 1.0f, v);
            Eng::template run<true>(a.pi, tws + salt, cs.t, cs.lds, v);
            z_store<Eng>(a, cs, pick3(a.out, oo), v);
        }
        return;
    }
    float2 *dst;
    if constexpr (MODE == ZM_ABSM) {
        // sa k^(y-2) FT(in0) + sb k^(y-1) FT(in1), one inverse transform
        const int cmid = Eng::out_count(a.pf, t);
        z_fwd_op<Eng, ZM_ABS>(a, c, 0, a.sa, v);
        float2 acc[E];
#pragma unroll
        for (int m = 0; m < E; ++m) acc[m] = v[m];
        z_load<Eng>(a, c, a.in[1], v);
        z_fwd_op<Eng, ZM_ABS>(a, c, 1, a.sb, v);
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cmid) v[m] = c_add(v[m], acc[m]);
        dst = a.out[0];
    } else {
        // (ABS: sa scales input 0, the tau term; 1 in the other modes)
        z_fwd_op<Eng, MODE>(a, c, o, (MODE == ZM_ABS && o == 0) ? a.sa : 1.0f, v);
        dst = pick3(a.out, o);
    }
    Eng::template run<true>(a.pi, tws, t, c.lds, v);
    z_store<Eng>(a, c, dst, v);
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
    int rho0_sum_in_z;       // density pass: the z pass forms FT(rho0 sum du) (constant rho0)
    float *rec_d[3];         // density pass, when recording a step for the reverse mode: the
    float *rec_rho[3];       // divergence components du_xi and the new rho_xi (else null)
    const float *rsrc;       // xfwd: real input
    float *rdst;             // xinv: real output
    float scale;
};

// c2r: packed spectrum row -> v[m] = x[2n] + i x[2n+1], n = out_index(pi, t, m)
// (unnormalised; the result is nx times the inverse DFT)
// S: the spectrum array; the row is row b of this block (rows of a block are
// consecutive: element k of it lies at a block-uniform address plus a lane
// offset, and M - k likewise).  UB = false: S differs between the lanes of a
// wavefront (thread groups of different fields), so plain per-lane pointers.
template <class Eng, bool UB = true>
__device__ __forceinline__ void row_c2r(const XArgs &a, const float2 *S, int b, bool ok,
                                        int t, const RowLds &lds, float2 (&v)[Eng::E],
                                        const float2 *twx, const float2 *twp, int salt = 0) {
    constexpr int E = Eng::E;
    const int M = a.g.M;
    const float2 *tw_post = twp + salt;
    const int cin = Eng::in_count(a.pi, t);
    if (ok) {
        const float2 *const blk = S + (size_t)blockIdx.x * a.tb * M;
        const int step = Eng::in_step(a.pi) + salt;   // (salt: see kw_xden)
        // k = t + m step: blk + m step + (b M + t);  M - k: blk + M - (m + 1) step + (b M + step - t)
        const uint32_t l1 = (uint32_t)(b * M + t) * 8u;
        const uint32_t l2 = (uint32_t)(b * M + step - t) * 8u;
        const float2 *const row = S + ((size_t)blockIdx.x * a.tb + b) * M;
        // every load first, then the arithmetic: with the k = 0 case as a
        // branch between the loads each element waited for its own loads
        // (k = 0 reads an element of its own row in place of M - k, unused)
        float2 P[E], Q[E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cin) {
                const int k = Eng::in_index(a.pi, t, m);
                if (UB) {
                    P[m] = ld_at(blk + m * step, l1);
                    Q[m] = ld_at(blk + M - (m + 1) * step, (m == 0 && t == 0) ? l2 - (uint32_t)step * 8u : l2);
                } else {
                    P[m] = row[k];
                    Q[m] = row[k == 0 ? 0 : M - k];
                }
            }
        }
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cin) {
                const int k = Eng::in_index(a.pi, t, m);
                const bool k0 = k == 0;
                const float2 xk = k0 ? make_float2(P[m].x, 0.0f) : P[m];
                const float2 xm = k0 ? make_float2(P[m].y, 0.0f) : Q[m];
                const float2 A = make_float2(xk.x + xm.x, xk.y - xm.y);        // xk + conj(xm)
                const float2 D = make_float2(xk.x - xm.x, xk.y + xm.y);        // xk - conj(xm)
                const float2 B = c_mulc(D, tw_post[k]);                         // * w^-k
                v[m] = make_float2(A.x - B.y, A.y + B.x);                       // A + i B
            }
        }
    }
    Eng::template run<true>(a.pi, twx + salt, t, lds, v);
}

// r2c: v[m] = x[2n] + i x[2n+1], n = in_index(pf, t, m)  ->  packed spectrum row
template <class Eng, bool UB = true>
__device__ __forceinline__ void row_r2c(const XArgs &a, float2 *S, int b, bool ok, int t,
                                        const RowLds &lds, float2 (&v)[Eng::E],
                                        const float2 *twx, const float2 *twp, int salt = 0) {
    constexpr int E = Eng::E;
    const int M = a.g.M;
    float2 *const blk = S + (size_t)blockIdx.x * a.tb * M;
    float2 *const row = S + ((size_t)blockIdx.x * a.tb + b) * M;
    const int ostep = Eng::out_step(a.pf);
    const uint32_t l1 = (uint32_t)(b * M + t) * 8u;
    const float2 *tw_post = twp + salt;
    Eng::template run<false>(a.pf, twx + salt, t, lds, v);
    const int cout = Eng::out_count(a.pf, t);
#pragma unroll
    for (int m = 0; m < E; ++m)
        if (m < cout) lds.st(Eng::out_index(a.pf, t, m), v[m]);
    lds.sync();
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
                if (UB) st_at(blk + m * ostep, l1, out);
                else row[k] = out;
            }
        }
    }
    lds.sync();
}

#define KW_XPROLOGUE                                                   \
    constexpr int E = Eng::E;                                          \
    extern __shared__ float2 lds_all[];                                \
    float2 *const tws = lds_all;          /* tw_x, then tw_post */     \
    float2 *const sh = lds_all + 2 * a.g.M;                            \
    stage_table(tws, a.t.tw_x, a.g.M);                                 \
    stage_table(tws + a.g.M, a.t.tw_post, a.g.M);                      \
    __syncthreads();                                                   \
    const int L = a.pf.L;                                              \
    const int tid = threadIdx.x, t = tid % L, b = tid / L;             \
    const int row = blockIdx.x * a.tb + b;                             \
    const bool ok = row < a.g.rows;                                    \
    const int rr = ok ? row : 0;                                       \
    const int M = a.g.M, nx = a.g.nx;                                  \
    const RowLds lds{sh, b * row_pitch(M), rows_in_waves(L)};          \
    const size_t rbase = (size_t)rr * nx;                              \
    const int cupd = Eng::out_count(a.pi, t);                          \
    /* real values x = 2 n, n = t + m step of row b: see XPos */       \
    const size_t xrow0 = (size_t)blockIdx.x * a.tb * nx;               \
    const uint32_t xlane = (uint32_t)(b * nx + 2 * t) * 4u;            \
    (void)nx; (void)rbase; (void)cupd; (void)xrow0; (void)xlane;

// Source values of the rows of this block, scattered into a per-row LDS line
// of nx floats (`fill` where there is no source point).  Returns whether the
// block has any source point (uniform over the block).
// Only threads with `worker` set fill the line (one group per row); every
// thread of the block takes the barriers.
__device__ __forceinline__ bool scatter_source(const XArgs &a, float *line, int row, bool ok,
                                               int t, int L, int b, bool worker = true,
                                               float fill = 0.0f) {
    const int nx = a.g.nx;
    int beg = 0, end = 0;
    if (a.src.row_ptr && ok && worker) {
        beg = a.src.row_ptr[row];
        end = a.src.row_ptr[row + 1];
    }
    const bool any = __syncthreads_or(end > beg);
    if (!any) return false;
    float *mine = line + (size_t)b * nx;
    if (worker)
        for (int x = t; x < nx; x += L) mine[x] = fill;
    __syncthreads();
    for (int e = beg + t; e < end; e += L)
        mine[a.src.xpos[e]] = a.src.coef[e] * a.src.drive[a.src.elem[e]];
    __syncthreads();
    return true;
}

// The three velocity components are independent: blockIdx.y selects one.
// FL bit 0: record u at the mask sensor points (the variant with the row
// scan); bit 1: a force source on one component.
enum { XV_USER = 1, XV_FORCE = 2 };
template <class Eng, int FL>
__global__ void __launch_bounds__(512) kw_xvel(XArgs a) {
    KW_XPROLOGUE
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const int xi = blockIdx.y;
    float2 v[E];
    // u, Delta t / rho0+ and the PML factors of the update are loaded before
    // the transform (independent of it): issued one element at a time between
    // the stores of the update, each waited for its own memory round trip.
    // Fixed engines up to 12 elements a thread: measured faster at 256^3,
    // 192^3 and 1024^3; the generic engines' register arrays went from five to
    // two wavefronts per SIMD with it (160^3 velocity pass 76 -> 100 us).
    constexpr bool PRE = Eng::fixed && Eng::E <= 12;
    float2 u0v[E], dv[E], qv[E];
    if constexpr (PRE) {
        float *u = pick3(a.fld, xi);
        const Coef dtr = xi == 0 ? a.m.dtr[0] : xi == 1 ? a.m.dtr[1] : a.m.dtr[2];
        const float qy = a.t.pml_sy[iy], qz = a.t.pml_sz[iz];
        if (ok) {
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m < cupd) {
                    const int x = 2 * Eng::out_index(a.pi, t, m);
                    const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                    u0v[m] = ld2(u, i);
                    if (xi == 0) qv[m] = *reinterpret_cast<const float2 *>(a.t.pml_sx + x);
                    else qv[m] = xi == 1 ? make_float2(qy, qy) : make_float2(qz, qz);
                }
            }
            if (dtr.map) {
#pragma unroll
                for (int m = 0; m < E; ++m)
                    if (m < cupd) dv[m] = ld2(dtr.map, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane});
            } else {
#pragma unroll
                for (int m = 0; m < E; ++m) dv[m] = make_float2(dtr.scalar, dtr.scalar);
            }
        }
    }
    row_c2r<Eng>(a, pick3(a.Sin, xi), b, ok, t, lds, v, tws, tws + M);
    // force source on this component: dt F per point in the LDS line
    float *const fline = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M)) + (size_t)b * nx;
    bool has_f = false;
    if constexpr ((FL & XV_FORCE) != 0) {
        if (xi == a.src.axis)                                        // block-uniform
            has_f = scatter_source(a, reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M)),
                                   rr, ok, t, L, b, true);
    }
    if (ok) {
        float *u = pick3(a.fld, xi);
        const Coef dtr = xi == 0 ? a.m.dtr[0] : xi == 1 ? a.m.dtr[1] : a.m.dtr[2];
        const float qy = a.t.pml_sy[iy], qz = a.t.pml_sz[iz];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const int x = 2 * Eng::out_index(a.pi, t, m);
                const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                float2 q, d, u0;
                if constexpr (PRE) {
                    q = qv[m];
                    d = dv[m];
                    u0 = u0v[m];
                } else {
                    if (xi == 0) q = make_float2(a.t.pml_sx[x], a.t.pml_sx[x + 1]);
                    else q = xi == 1 ? make_float2(qy, qy) : make_float2(qz, qz);
                    d = coef2_at(dtr, i);
                    u0 = ld2(u, i);
                }
                const float2 g = v[m];
                float2 un;
                un.x = q.x * (q.x * u0.x - d.x * g.x);
                un.y = q.y * (q.y * u0.y - d.y * g.y);
                if constexpr ((FL & XV_FORCE) != 0) {
                    if (has_f) {
                        un.x += fline[x];
                        un.y += fline[x + 1];
                    }
                }
                st2(u, i, un);
                v[m] = un;
            }
        }
    }
    if constexpr ((FL & XV_USER) != 0) {
        // u^(n+1/2) is recorded with p^(n+1): step counter n + 1, already advanced
        const int step = *a.cnt.step;
        const int slot = step - a.sen.record_start;
        if (step >= a.sen.record_start && slot < a.sen.capacity) {
            int beg = 0, end = 0;
            if (ok) {
                beg = a.sen.row_ptr[rr];
                end = a.sen.row_ptr[rr + 1];
            }
            if (__syncthreads_or(end > beg)) {
                float *mine = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M)) + (size_t)b * nx;
                if (ok) {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        if (m < cupd) {
                            const int x = 2 * Eng::out_index(a.pi, t, m);
                            mine[x] = v[m].x;
                            mine[x + 1] = v[m].y;
                        }
                    }
                }
                __syncthreads();
                for (int e = beg + t; e < end; e += L)
                    a.sen.u_series[((size_t)slot * 3 + xi) * a.sen.n_points + a.sen.sid[e]] =
                        mine[a.sen.xpos[e]];
                __syncthreads();
            }
        }
    }
    row_r2c<Eng>(a, pick3(a.Sout, xi), b, ok, t, lds, v, tws, tws + M);
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
        if (a.sen.p_min) a.sen.p_min[id] = fminf(a.sen.p_min[id], pv);
        if (a.sen.p_sum2) a.sen.p_sum2[id] += pv * pv;
        if (a.sen.series && slot < a.sen.capacity)
            a.sen.series[(size_t)slot * a.sen.n_points + id] = pv;
        for (int h = 0; h < a.sen.n_harm; ++h) {
            // p e^{-i h w t}
            float2 *acc = reinterpret_cast<float2 *>(a.sen.harm) + (size_t)h * a.sen.n_points + id;
            const float c = a.sen.hw[2 * h], sn = a.sen.hw[2 * h + 1];
            *acc = make_float2(acc->x + pv * c, acc->y - pv * sn);
        }
    }
    __syncthreads();
}

// sensors, non-finite check and x r2c of the new pressure (v holds p in the
// output layout of the inverse x transform)
// SENS: the rarer sensor work is compiled in (mask sensors, p_min, harmonic
// sums); without it the register count of the common case stays lower
template <class Eng, bool SENS = true>
__device__ __forceinline__ void finish_pressure(const XArgs &a, float *line, int row, bool ok,
                                                int t, int L, int b, const RowLds &lds,
                                                float2 (&v)[Eng::E], const float2 *twx,
                                                const float2 *twp) {
    constexpr int E = Eng::E;
    const int M = a.g.M, nx = a.g.nx;
    const size_t rbase = (size_t)(ok ? row : 0) * nx;
    const size_t xrow0 = (size_t)blockIdx.x * a.tb * nx;
    const uint32_t xlane = (uint32_t)(b * nx + 2 * t) * 4u;
    const int step = *a.cnt.step;
    const bool rec = step >= a.sen.record_start;
    const int cnt = Eng::out_count(a.pi, t);
    if constexpr (SENS) {
        // pressure source: p^(n+1) = s at the source points (NaN marks the others)
        if (a.src.row_ptr && a.src.kind == KW_SOURCE_PRESSURE &&
            scatter_source(a, line, row, ok, t, L, b, true, __builtin_nanf(""))) {
            const float *mine = line + (size_t)b * nx;
            if (ok) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    if (m < cnt) {
                        const int x = 2 * Eng::out_index(a.pi, t, m);
                        const float s0 = mine[x], s1 = mine[x + 1];
                        if (s0 == s0) v[m].x = s0;
                        if (s1 == s1) v[m].y = s1;
                    }
                }
            }
            __syncthreads();
        }
    }
    bool bad = false;
    if (ok && rec && a.sen.all_points) {
        // each accumulator: every element's load, then every store (stored one
        // element at a time between the loads, each element waited for its
        // own load: the stores might alias the next loads)
        if (a.sen.p_max) {
            float2 acc[E];
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cnt) acc[m] = ld2(a.sen.p_max, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane});
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cnt)
                    st2(a.sen.p_max, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane},
                        make_float2(fmaxf(acc[m].x, v[m].x), fmaxf(acc[m].y, v[m].y)));
        }
        if (a.sen.p_sum2) {
            float2 acc[E];
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cnt) acc[m] = ld2(a.sen.p_sum2, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane});
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cnt)
                    st2(a.sen.p_sum2, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane},
                        make_float2(acc[m].x + v[m].x * v[m].x, acc[m].y + v[m].y * v[m].y));
        }
    }
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cnt) {
                const float2 p = v[m];
                bad |= !(__builtin_isfinite(p.x) && __builtin_isfinite(p.y));
                if (rec && a.sen.all_points) {
                    const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                    if constexpr (SENS) {
                        if (a.sen.p_min) {
                            const float2 mn = ld2(a.sen.p_min, i);
                            st2(a.sen.p_min, i, make_float2(fminf(mn.x, p.x), fminf(mn.y, p.y)));
                        }
                        const size_t nrec = (size_t)a.g.nx * a.g.rows;
                        const size_t ix = rbase + 2 * Eng::out_index(a.pi, t, m);
                        for (int h = 0; h < a.sen.n_harm; ++h) {
                            // points ix, ix+1: (re, im) pairs of p e^{-i h w t}
                            float4 *acc = reinterpret_cast<float4 *>(a.sen.harm + 2 * ((size_t)h * nrec + ix));
                            const float c = a.sen.hw[2 * h], sn = a.sen.hw[2 * h + 1];
                            const float4 o = *acc;
                            *acc = make_float4(o.x + p.x * c, o.y - p.x * sn, o.z + p.y * c,
                                               o.w - p.y * sn);
                        }
                    }
                }
            }
        }
    }
    if (bad) atomicMin(a.cnt.nonfinite, step);
    if constexpr (SENS) {
        if (rec && !a.sen.all_points && a.sen.row_ptr)
            record_mask<Eng>(a, line, row, ok, t, L, b, step, v);
    }
    row_r2c<Eng>(a, a.Sout[0], b, ok, t, lds, v, twx, twp);
}

// Density update (Eqs. (4c), (8) with the split-field PML of Eq. (6)), and
// what follows from rho within the step.  One thread group per row (as in
// kw_xvel) runs the three split components one after the other -- inverse x
// transform of du_xi, update of rho_xi -- and keeps the sums over the
// components in registers: sum rho (rho, stored for the pressure kernel) and
// sum du.  With absorption it then transforms rho0 sum du (into Sout[0]) and
// rho (into Sout[1]) for the absorption pass; without, it evaluates the
// equation of state and finishes the pressure like kw_xeos.
// The transforms of a row synchronise only its wavefront (RowLds), so the
// wavefronts of a block run independently between the few block barriers
// (twiddle staging, the source scatter, sensors).
// SRC: a mass source (values scattered once into the still idle FFT buffers
// and kept in registers); ABS = a.m.absorbing.  Both are template parameters
// so that the common paths do not carry the registers of the others.
template <class Eng, bool ABS, bool SRC>
__global__ void __launch_bounds__(512) kw_xden(XArgs a) {
    KW_XPROLOGUE
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const float dt = a.g.dt;
    // source values and sensor lines alias the FFT buffers; every use lies
    // between block barriers, outside the transforms
    float *const line = reinterpret_cast<float *>(sh);
    float2 sv[SRC ? E : 1];
    bool has_src = false;
    if constexpr (SRC) {
        has_src = scatter_source(a, line, rr, ok, t, L, b);
        if (has_src) {
            const float *mine = line + (size_t)b * nx;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int x = 2 * Eng::out_index(a.pi, t, m);
                sv[m] = (m < cupd) ? make_float2(mine[x], mine[x + 1]) : make_float2(0.f, 0.f);
            }
            __syncthreads();
        }
    }
    float2 sr[E], sd[ABS ? E : 1];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        sr[m] = make_float2(0.f, 0.f);
        if constexpr (ABS) sd[m] = make_float2(0.f, 0.f);
    }
    const float qy = a.t.pml_y[iy], qz = a.t.pml_z[iz];
    // a rho0 map is read from HBM once: the first component keeps the row's
    // values in an LDS line (each thread reads back only what it wrote), where
    // the others and the final product find them; reading it four times from
    // global memory fetched 2.3 extra units per point, the block's lines
    // having left L2 by the next component
    const bool r0map = a.m.rho0.map != nullptr;
    float *const r0l = reinterpret_cast<float *>(sh + (size_t)a.tb * row_pitch(M)) + (size_t)b * nx;
#pragma unroll 1
    for (int g = 0; g < 3; ++g) {
        // salt = 0, unknown to the compiler: it makes the element indices
        // depend on g, so that they are recomputed in every iteration rather
        // than hoisted out of the loop and held in registers across it
        const int salt = g * a.zero;
        const int ts = t + salt;
        const RowLds ldg{sh, lds.base + salt, lds.wave};
        float2 v[E];
        row_c2r<Eng>(a, pick3(a.Sin, g), b, ok, ts, ldg, v, tws, tws + M, salt);
        float *rho = pick3(a.fld, g);
        // rho_xi of every element loaded before the updates (between the
        // stores of the previous elements each load waited for itself)
        float2 oldv[E];
        if (ok) {
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cupd)
                    oldv[m] = ld2(rho, XPos{xrow0 + 2 * (size_t)m * (Eng::out_step(a.pi) + salt),
                                            (uint32_t)(b * nx + 2 * ts) * 4u});
        }
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
                    float2 r0;
                    if (!r0map) {
                        r0 = make_float2(a.m.rho0.scalar, a.m.rho0.scalar);
                    } else if (g == 0) {
                        r0 = ld2(a.m.rho0.map, i);
                        *reinterpret_cast<float2 *>(r0l + x) = r0;
                    } else {
                        r0 = *reinterpret_cast<const float2 *>(r0l + x);
                    }
                    const float2 old = oldv[m];
                    const float2 d = v[m];
                    float2 nw;
                    nw.x = q.x * (q.x * old.x - dt * r0.x * d.x);
                    nw.y = q.y * (q.y * old.y - dt * r0.y * d.y);
                    if (a.m.nonlinear) {
                        // the denominator of Eq. (4d) is 1 + O(dt du): the hardware
                        // reciprocal (1 ulp) replaces the IEEE division sequence
                        nw.x *= __builtin_amdgcn_rcpf(1.0f + 2.0f * dt * d.x);
                        nw.y *= __builtin_amdgcn_rcpf(1.0f + 2.0f * dt * d.y);
                    }
                    if constexpr (SRC) {
                        if (has_src) nw = c_add(nw, sv[m]);
                    }
                    st2(rho, i, nw);
                    if (a.rec_d[0]) {                    // block-uniform
                        st2(pick3(a.rec_d, g), i, d);
                        st2(pick3(a.rec_rho, g), i, nw);
                    }
                    sr[m] = c_add(sr[m], nw);
                    if constexpr (ABS) sd[m] = c_add(sd[m], d);
                }
            }
        }
    }
    float2 v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        v[m] = make_float2(0.f, 0.f);
        if (m < cupd && ok) {
            const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
            const float2 r = sr[m];
            if constexpr (ABS) {
                const float2 r0 = r0map ? *reinterpret_cast<const float2 *>(r0l + 2 * Eng::out_index(a.pi, t, m))
                                        : make_float2(a.m.rho0.scalar, a.m.rho0.scalar);
                v[m] = make_float2(r0.x * sd[m].x, r0.y * sd[m].y);
                st2(a.rho_total, i, r);
            } else {
                const float2 c2 = coef2_at(a.m.c0sq, i);
                float2 pp = make_float2(c2.x * r.x, c2.y * r.y);
                if (a.m.nonlinear) {
                    const float2 nl = coef2_at(a.m.nl, i);
                    pp.x += nl.x * r.x * r.x;
                    pp.y += nl.y * r.y * r.y;
                }
                v[m] = pp;
            }
        }
    }
    if constexpr (ABS) {
        // (with a constant rho0 the divergence pass forms the spectrum of
        // rho0 sum du itself: only rho is transformed here)
        if (!a.rho0_sum_in_z) row_r2c<Eng>(a, a.Sout[0], b, ok, t, lds, v, tws, tws + M);
        row_r2c<Eng>(a, a.Sout[1], b, ok, t, lds, sr, tws, tws + M);
    } else {
        finish_pressure<Eng>(a, line, rr, ok, t, L, b, lds, v, tws, tws + M);
    }
}

// Density update for the generic engines, whose register arrays are sized for
// their largest radix (sums of three components in registers, as kw_xden
// keeps them, would cost two more such arrays).  The three split components are coupled only through
// rho = sum rho_xi and sum du_xi, so a block runs them side by side: thread
// group g (g = 0, 1, 2) transforms and updates component g of the block's tb
// rows, and then group 0 transforms rho0 sum du and group 1 stores rho and
// transforms it (group 2 takes the same barriers without storing).  Without
// absorption group 1 evaluates the equation of state instead.  Each thread
// holds one component's values, as in kw_xvel.
// The groups exchange only what the others need: group 0 keeps du_0 and group
// 1 keeps rho_1 in registers; rho_0, du_1 and rho_2 go to the (then idle) FFT
// buffers of groups 0, 1 and 2, and du_2 to a line of its own.
// LDS: [3 groups][tb rows] FFT buffers, [tb] du_2 lines (twiddles during the transforms),
// [tb] source lines.
// ABS (= a.m.absorbing) is a template parameter: the lossless tail (equation
// of state, sensors, pressure transform) would otherwise set the register
// count of the absorbing kernel too.
template <class Eng, bool ABS>
__global__ void __launch_bounds__(512) kw_xden3(XArgs a) {
    constexpr int E = Eng::E;
    extern __shared__ float2 lds_all[];
    float2 *const sh = lds_all;
    const int L = a.pf.L;
    const int M = a.g.M, nx = a.g.nx, tb = a.tb;
    const int tid = threadIdx.x;
    const int g = tid / (tb * L);
    const int rem = tid - g * tb * L;
    const int b = rem / L, t = rem % L;
    const int row = blockIdx.x * tb + b;
    const bool ok = row < a.g.rows;
    const int rr = ok ? row : 0;
    const int iy = rr % a.g.ny, iz = rr / a.g.ny;
    const size_t rbase = (size_t)rr * nx;
    const int RP = row_pitch(M);
    // block barriers in the transforms: the exchange below and the twiddles
    // in the du_2 lines need every group past its transform
    const RowLds lds{sh, (g * tb + b) * RP, false};
    float2 *buf0 = sh + (size_t)b * RP;                      // row b's buffer of group 0
    float2 *buf1 = sh + (size_t)(tb + b) * RP;
    float2 *buf2 = sh + (size_t)(2 * tb + b) * RP;
    float2 *du2 = sh + (size_t)3 * tb * RP + (size_t)b * M;   // nx floats per row
    float *line = reinterpret_cast<float *>(sh + (size_t)3 * tb * RP + (size_t)tb * M);
    // The twiddle tables (tw_x, and tw_post when there are two lines or more)
    // are staged in the du_2 lines, which are free during both transforms:
    // once for the inverse transforms of phase 1 (du_2 is written after them)
    // and again for the forward transforms of phase 2 (after du_2 has been
    // read).  This keeps the LDS of three 10-row blocks within a CU.
    float2 *const tws = sh + (size_t)3 * tb * RP;
    const bool post_lds = tb >= 2;                                    // block-uniform
    const float2 *const twp = post_lds ? tws + M : a.t.tw_post;
    stage_table(tws, a.t.tw_x, M);
    if (post_lds) stage_table(tws + M, a.t.tw_post, M);
    __syncthreads();
    const float dt = a.g.dt;
    const int cupd = Eng::out_count(a.pi, t);

    const bool has_src = a.src.kind == KW_SOURCE_MASS &&
                         scatter_source(a, line, rr, ok, t, L, b, g == 0);
    const float *mysrc = line + (size_t)b * nx;

    // phase 1: component g (row_c2r ends with a barrier, so the FFT buffers
    // are free for the exchange afterwards)
    float2 v[E];
    row_c2r<Eng, false>(a, pick3(a.Sin, g), b, ok, t, lds, v, tws, twp);
    {
        float *rho = pick3(a.fld, g);
        const float qy = a.t.pml_y[iy], qz = a.t.pml_z[iz];
        float2 *xrho = (g == 0) ? buf0 : buf2;
        // rho_g of every element loaded before the updates (between the
        // stores of the previous elements each load waited for itself); the
        // fixed engines only (measured: 192^3 density pass 155 -> 152 us, the
        // generic engine's 160^3 one 86 -> 93 us for a wavefront less)
        constexpr bool PRE = Eng::fixed && Eng::E <= 12;
        float2 oldv[E];
        if (PRE && ok) {
#pragma unroll
            for (int m = 0; m < E; ++m)
                if (m < cupd) oldv[m] = ld2(rho, rbase + 2 * Eng::out_index(a.pi, t, m));
        }
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const int n = Eng::out_index(a.pi, t, m);
                const int x = 2 * n;
                const size_t i = rbase + x;
                float2 nw = make_float2(0.0f, 0.0f);
                const float2 d = v[m];
                if (ok) {
                    float2 q;
                    if (g == 0) q = make_float2(a.t.pml_x[x], a.t.pml_x[x + 1]);
                    else if (g == 1) q = make_float2(qy, qy);
                    else q = make_float2(qz, qz);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    const float2 old = PRE ? oldv[m] : ld2(rho, i);
                    nw.x = q.x * (q.x * old.x - dt * r0.x * d.x);
                    nw.y = q.y * (q.y * old.y - dt * r0.y * d.y);
                    if (a.m.nonlinear) {
                        nw.x *= __builtin_amdgcn_rcpf(1.0f + 2.0f * dt * d.x);
                        nw.y *= __builtin_amdgcn_rcpf(1.0f + 2.0f * dt * d.y);
                    }
                    if (has_src) {
                        nw.x += mysrc[x];
                        nw.y += mysrc[x + 1];
                    }
                    st2(rho, i, nw);
                    if (a.rec_d[0]) {                    // block-uniform
                        st2(pick3(a.rec_d, g), i, d);
                        st2(pick3(a.rec_rho, g), i, nw);
                    }
                }
                if (g == 1) {
                    buf1[n] = d;
                    v[m] = nw;
                } else {
                    xrho[n] = nw;
                    if (g == 2) du2[n] = d;
                }
            }
        }
    }
    __syncthreads();

    // phase 2: sums over the components (group 0: sum du, group 1: rho)
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (m < cupd) {
            const int n = Eng::out_index(a.pi, t, m);
            const size_t i = rbase + 2 * n;
            if (g == 0) {
                if constexpr (ABS) {
                    const float2 s = c_add(c_add(v[m], buf1[n]), du2[n]);
                    const float2 r0 = coef2_at(a.m.rho0, i);
                    v[m] = make_float2(r0.x * s.x, r0.y * s.y);
                }
            } else if (g == 1) {
                const float2 r = c_add(c_add(v[m], buf0[n]), buf2[n]);
                if constexpr (ABS) {
                    v[m] = r;
                    if (ok) st2(a.rho_total, i, r);
                } else {
                    const float2 c2 = coef2_at(a.m.c0sq, i);
                    float2 pp = make_float2(c2.x * r.x, c2.y * r.y);
                    if (a.m.nonlinear) {
                        const float2 nl = coef2_at(a.m.nl, i);
                        pp.x += nl.x * r.x * r.x;
                        pp.y += nl.y * r.y * r.y;
                    }
                    v[m] = pp;
                }
            }
        }
    }
    __syncthreads();   // the forward transforms below overwrite the exchanged values
    stage_table(tws, a.t.tw_x, M);
    if (post_lds) stage_table(tws + M, a.t.tw_post, M);
    __syncthreads();
    if constexpr (ABS) {
        float2 *dst = (g == 0) ? a.Sout[0] : a.Sout[1];
        const bool out = g == 1 || (g == 0 && !a.rho0_sum_in_z);
        row_r2c<Eng, false>(a, dst, b, ok && out, t, lds, v, tws, twp);
    } else {
        finish_pressure<Eng>(a, line, rr, ok && g == 1, t, L, b, lds, v, tws, twp);
    }
}

// SENS: mask sensors, p_min or harmonic sums are recorded (see finish_pressure)
// MERGED: one input spectrum that already holds ta a + tb b (merged absorption
// pass of a medium with scalar ta, tb) instead of a and b.
// Asked to fit six wavefronts per SIMD (80 registers; a few bytes spill):
// measured faster than five without spills.  The wider engines would spill
// hundreds of bytes at 80 registers: no request for them.
// The sensor and pressure-source lines alias the FFT row buffers (nx floats a
// row fit in a buffer of row_pitch(M) complex values): they are used only
// between the inverse transforms and the forward one, behind block barriers.
template <class Eng, bool SENS, bool MERGED>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((Eng::fixed && Eng::E <= 8) ? 6 : 1)))
kw_xeos(XArgs a) {
    KW_XPROLOGUE
    float *line = reinterpret_cast<float *>(sh);
    float2 va[E], v[E];
    if constexpr (!MERGED)
        row_c2r<Eng>(a, a.Sin[0], b, ok, t, lds, va, tws, tws + M);
    row_c2r<Eng>(a, a.Sin[MERGED ? 0 : 1], b, ok, t, lds, v, tws, tws + M);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m < cupd) {
                const XPos i{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane};
                const float2 rho = ld2(a.rho_total, i);
                const float2 c2 = coef2_at(a.m.c0sq, i);
                float2 p;
                if constexpr (MERGED) {
                    p.x = c2.x * rho.x + v[m].x;
                    p.y = c2.y * rho.y + v[m].y;
                } else {
                    const float2 ta = coef2_at(a.m.ta, i);
                    const float2 tb = coef2_at(a.m.tb, i);
                    p.x = c2.x * rho.x + ta.x * va[m].x + tb.x * v[m].x;
                    p.y = c2.y * rho.y + ta.y * va[m].y + tb.y * v[m].y;
                }
                if (a.m.nonlinear) {
                    const float2 nl = coef2_at(a.m.nl, i);
                    p.x += nl.x * rho.x * rho.x;
                    p.y += nl.y * rho.y * rho.y;
                }
                v[m] = p;
            }
        }
    }
    finish_pressure<Eng, SENS>(a, line, rr, ok, t, L, b, lds, v, tws, tws + M);
}

template <class Eng>
__global__ void __launch_bounds__(512) kw_xfwd(XArgs a) {
    KW_XPROLOGUE
    float2 v[E];
    const int cin = Eng::in_count(a.pf, t);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cin) v[m] = ld2(a.rsrc, XPos{xrow0 + 2 * (size_t)m * Eng::in_step(a.pf), xlane});
    }
    row_r2c<Eng>(a, a.Sout[0], b, ok, t, lds, v, tws, tws + M);
}

template <class Eng>
__global__ void __launch_bounds__(512) kw_xinv(XArgs a) {
    KW_XPROLOGUE
    float2 v[E];
    row_c2r<Eng>(a, a.Sin[0], b, ok, t, lds, v, tws, tws + M);
    if (ok) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (m < cupd)
                st2(a.rdst, XPos{xrow0 + 2 * (size_t)m * Eng::out_step(a.pi), xlane}, c_scale(v[m], a.scale));
    }
}

// engine dispatch ---------------------------------------------------------------
#define KW_ENGINE_SWITCH(ENG, BODY)                                            \
    switch (ENG) {                                                             \
    case ENG_G16: { using Eng = EngGeneric<16>; BODY; } break;                 \
    case ENG_G32: { using Eng = EngGeneric<32>; BODY; } break;                 \
    case ENG_F4:  { using Eng = EngFixed<4>; BODY; } break;                    \
    case ENG_F8:  { using Eng = EngFixed<8>; BODY; } break;                    \
    case ENG_F8P: { using Eng = EngFixed8P; BODY; } break;              \
    case ENG_F8_84: { using Eng = EngFixed8_84; BODY; } break;          \
    case ENG_F16P: { using Eng = EngFixed16P; BODY; } break;            \
    case ENG_F12: { using Eng = EngFixed<12>; BODY; } break;                   \
    case ENG_F12_64: { using Eng = EngFixed12_64; BODY; } break;               \
    case ENG_F20: { using Eng = EngFixed<20>; BODY; } break;                   \
    case ENG_F32: { using Eng = EngFixed<32>; BODY; } break;                   \
    default:      { using Eng = EngFixed<16>; BODY; } break;                   \
    }

}  // namespace kw
