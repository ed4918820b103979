// Internal structures shared by the host engine (engine.cpp) and the HIP
// kernels (kernels_*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kw.h"

namespace kw {

constexpr int kMaxPasses = 8;

// Radix schedule of one 1D transform.  Passes run in the listed order.  With
// the generic engine the inverse transform of an axis uses the factors in
// reverse order, so that the last inverse pass and the first forward pass
// share one register layout; the fixed-width engine has the same layout for
// every plan.  Either way an inverse FFT, an element-wise update and a forward
// FFT run back to back without an LDS exchange in between.
struct FftPlan {
    int n;                    // transform length (complex points)
    int np;                   // number of passes
    int L;                    // threads per transform (generic: max n / radix; fixed: n / E)
    int rmax;                 // largest radix
    unsigned long long code;  // radix of pass p in bits [6p, 6p + 6): read on the device
                              // without indexing an array (a run-time index into a
                              // by-value kernel argument would move it to scratch)
    int radix[kMaxPasses];    // host copy of the same schedule
};

__host__ __device__ inline int plan_radix(const FftPlan &P, int p) {
    return (int)((P.code >> (6 * p)) & 63ull);
}

// One real field or spectrum array plus an optional per-point map: when
// `map` is null the scalar is used everywhere.
struct Coef {
    const float *map;
    float scalar;
};

struct GridDev {
    int nx, ny, nz;          // real grid
    int M;                   // nx / 2: complex points per packed half-spectrum row
    int rows;                // ny * nz
    float inv_n;             // 1 / (nx ny nz)
    float half_cdt;          // c_ref * dt / 2 (argument scale of kappa)
    float dt;
    float y_tau;             // (y - 2) / 2, exponent of k^2 for k^(y-2)
    float y_eta;             // (y - 1) / 2
    float dkz;               // 2 pi / (nz dz): kz of FFT index m is m dkz (Eq. (5))
};

// 1D tables (device), float32 copies of float64 host values.
struct Tables {
    const float2 *tw_x;      // exp(-2 pi i m / M), m < M
    const float2 *tw_post;   // exp(-2 pi i k / nx), k < M  (real-FFT split twiddles)
    const float2 *tw_y;      // exp(-2 pi i m / ny)
    const float2 *tw_z;      // exp(-2 pi i m / nz)
    const float *kx;         // [M + 1]  (index M is the Nyquist wavenumber -pi/dx)
    const float *ky;         // [ny]
    const float *kz;         // [nz]
    const float2 *dpx, *dmx; // [M + 1]  i kx exp(+- i kx dx / 2)
    const float2 *dpy, *dmy; // [ny]
    const float2 *dpz, *dmz; // [nz]
    const float *pml_x, *pml_sx;   // [nx] regular / staggered PML factors
    const float *pml_y, *pml_sy;   // [ny]
    const float *pml_z, *pml_sz;   // [nz]
};

struct SourceDev {
    int n_elements;
    const int *row_ptr;      // [rows + 1] CSR over grid rows (null -> no source)
    const int *xpos;         // x of each source point
    const int *elem;         // element of each point
    const float *coef;       // 2 dt / (3 c0 dx) at each point
    const double *amp_cos;   // a_e cos(phi_e)
    const double *amp_sin;   // a_e sin(phi_e)
    const float *signal;     // optional [n_elements * n_samples]
    int n_samples;
    double omega_dt;         // 2 pi f dt
    float *drive;            // [n_elements] value of s_e in the current step
    int kind;                // KW_SOURCE_* (mass, force, pressure)
    int axis;                // velocity component of a force source
    double t_offset;         // drive time of step n: (n + t_offset) dt
};

struct SensorDev {
    int all_points;          // 1 -> one accumulator per grid point
    int n_points;
    const int *row_ptr;      // [rows + 1] CSR (mask mode)
    const int *xpos;
    const int *sid;          // sensor id (position in the sorted index list)
    float *p_max;            // null when not recorded
    float *p_sum2;           // null when neither p_rms nor intensity is recorded
    float *series;           // [capacity * n_points] or null
    int capacity;
    int record_start;
    float *p_min;            // null when not recorded
    float *harm;             // [n_harm][points][2] running sums of p e^{-i h w t}, or null
    float *hw;               // [n_harm][2] cos, sin of h w t for the step being recorded
    int n_harm;
    double harm_wdt;         // 2 pi f dt of the harmonic base frequency
    float *u_series;         // [capacity][3][n_points] or null
};

struct Medium {
    Coef dtr[3];             // dt / rho0 at the staggered points of u_x, u_y, u_z
    Coef rho0;               // rho0
    Coef c0sq;               // c0^2
    Coef nl;                 // c0^2 B/A / (2 rho0)            (nonlinear)
    Coef ta;                 // c0^2 tau                        (absorbing)
    Coef tb;                 // -c0^2 eta                       (absorbing)
    int nonlinear;
    int absorbing;
};

struct Counters {
    int *step;               // steps taken (device)
    int *nonfinite;          // first step with a non-finite pressure (INT_MAX if none)
};

// kernel launch records -------------------------------------------------------
enum KernelClass {
    KC_YFWD = 0, KC_YINV, KC_ZGRAD, KC_ZDIV, KC_ZABS,
    KC_XVEL, KC_XDEN, KC_XEOS, KC_COUNT
};

struct StepBuffers {
    float *u[3];
    float *rho[3];
    float *rho_total;        // sum of the split densities (absorbing only)
    float2 *S[7];            // packed half-spectrum scratch arrays
};

// FFT engines: generic one-butterfly-per-thread Stockham with register arrays
// of 16 or 32 (any 2^a 3^b 5^c length), or the fixed-width engine with 8 or 16
// elements per thread (power-of-two lengths, radices 2/4/8/16).
// ENG_F8P, ENG_F16P: the 8- and 16-wide fixed engines for plans whose passes
// all have radix 8 (16); ENG_F8_84: the 8-wide one for plans of radices 8
// and 4; ENG_F12_64: the 12-wide one for plans of radices 6 and 4.  The
// kernels built for a set of radices hold fewer registers.
enum EngId { ENG_G16 = 0, ENG_G32 = 1, ENG_F8 = 2, ENG_F16 = 3, ENG_F4 = 4, ENG_F12 = 5, ENG_F20 = 6,
             ENG_F32 = 7, ENG_F8P = 8, ENG_F16P = 9, ENG_F12_64 = 10, ENG_F8_84 = 11 };
// the engine of the same width that runs any plan (ENG_F8P -> ENG_F8, ...)
inline int eng_general(int e) {
    return (e == ENG_F8P || e == ENG_F8_84) ? ENG_F8 : e == ENG_F16P ? ENG_F16
         : e == ENG_F12_64 ? ENG_F12 : e;
}
inline bool eng_fixed(int e) {
    e = eng_general(e);
    return e == ENG_F4 || e == ENG_F8 || e == ENG_F16 || e == ENG_F12 || e == ENG_F20 || e == ENG_F32;
}
// fixed engines whose register arrays are too wide for the kernels that keep
// a second spectrum or sums per thread (they take the generic engines' paths)
inline bool eng_wide(int e) { return e == ENG_F20 || e == ENG_F32; }

struct LaunchCfg {
    int eng_x, eng_y, eng_z; // EngId per axis
    FftPlan px, pxi;         // x forward plan (length M) and the plan of the inverse
    FftPlan py, pyi;         // y
    FftPlan pz, pzi;         // z
    int tb_x;                // rows per block in x kernels
    int tb_den;              // rows per block of the three-group density kernel (generic engines)
    int tb_y;                // columns per block in y kernels
    int tb_z;                // columns per block in z kernels
    int eng_za;              // the merged absorption z pass: engine, plans and
    FftPlan pza, pzai;       // columns per block (the z pass's own unless a
    int tb_za;               // better one is known for its length)
};

// LDS of the three-group density kernel (generic engines): the FFT buffers
// of its 3 thread groups, a line of nx floats per row for du of component z,
// and, when `line`, one more for source values (or mask sensor values in the
// lossless case)
inline bool den_needs_line(const Medium &m, const SourceDev &src, const SensorDev &sen) {
    // a mass source, or (lossless: the density kernel ends with the pressure)
    // mask sensors or a pressure source
    return (src.row_ptr != nullptr && src.kind == KW_SOURCE_MASS) ||
           (!m.absorbing && ((sen.row_ptr != nullptr && !sen.all_points) ||
                             (src.row_ptr != nullptr && src.kind == KW_SOURCE_PRESSURE)));
}
// LDS pitch (complex values) of a row buffer of the x passes: n values plus
// one pad slot per 16 (see RowLds)
__host__ __device__ inline int row_pitch(int n) { return n + (n >> 4) + 1; }
inline size_t den_lds_bytes(int M, int nx, int tb, bool line) {
    const size_t rp = (size_t)row_pitch(M);
    return (size_t)3 * tb * rp * 8 + (size_t)tb * M * 8 +
           (line ? (size_t)tb * nx * 4 : 0);
}
// LDS of the x kernels (twiddle tables, one FFT row buffer per row, and
// optionally a line of nx floats per row), of the y pass and of the z pass
// (twiddle table and the column tile)
inline size_t x_lds_bytes(int M, int nx, int tb, bool line) {
    const size_t rp = (size_t)row_pitch(M);
    return (size_t)2 * M * 8 + (size_t)tb * rp * 8 + (line ? (size_t)tb * nx * 4 : 0);
}
inline size_t col_lds_bytes(int n, int tb) { return (size_t)n * 8 + (size_t)tb * n * 8; }
// the z pass keeps two tables of nz entries (twiddles, z factors) before its tile
__host__ __device__ inline int zpass_table_slots(int nz) { return 2 * nz; }
inline size_t zcol_lds_bytes(int n, int tb) {
    return (size_t)zpass_table_slots(n) * 8 + (size_t)tb * n * 8;
}

// GRAD: one input, output o multiplied by D+_o kappa / N          (Eq. (4a))
// DIV:  input o, output o multiplied by D-_o kappa / N            (Eq. (4c))
// ABS:  input o multiplied by k^(y-2) / N (o = 0), k^(y-1) / N     (Eq. (8))
// DIVT, GRADT: input o, output o multiplied by conj(D-_o kappa) / N and
// conj(D+_o kappa) / N, the transposes of the real operators of DIV and GRAD
// (used by the reverse-mode step)
// ABSM: ta k^(y-2) / N on input 0 plus tb k^(y-1) / N on input 1, summed into
// one output (the two absorption terms of Eq. (8) for a medium whose
// c0^2 tau and c0^2 eta are scalars: one inverse transform instead of two)
// ABS and ABSM take an optional pair of addends of input 0 (add0): with a
// constant rho0 input 0 is then the sum of the three divergence outputs, and
// sa carries rho0 nx ny (see enqueue_step)
enum { ZM_GRAD = 0, ZM_DIV = 1, ZM_ABS = 2, ZM_DIVT = 3, ZM_GRADT = 4, ZM_ABSM = 5 };

// reverse-mode (adjoint) step state, all device arrays of N floats unless noted
struct AdjDev {
    float *pb;               // adjoint of p^(n+1) (carried between reverse steps)
    float *ub[3];            // adjoint of u^(n+1/2)
    float *rb[3];            // adjoint of rho_xi^(n+1)
    float *d[3];             // adjoint of the divergence d_xi (the forward d_xi first, when
                             // it is recomputed rather than read from a step record)
    const float *dfw[3];     // forward divergence d_xi of the step being reversed
    const float *rho[3];     // forward rho_xi after that step
    float *w;                // 2 w / (rho0 c0 N_w): derivative of the objective
    float *rbt;              // adjoint of rho (the sum of the components)
    double *dJds;            // [n_steps][n_elements] derivative by the drive values
    double *obj;             // objective J (one value)
    int n_steps, n_elem;
    int n_src;               // source points
    const int *src_flat;     // flat index, element and coefficient of each point
    const int *src_elem;
    const float *src_coef;
    float *add;              // [n_src] drive term coef_k s_e(n) of each point in this step
    float *rsrc;             // [3][n_src] R_xi at each source point (see kw_adjx_den)
    const int *elem_ptr;     // [n_elem + 1] CSR of the points of each element
    const int *elem_pts;     // point numbers (k) of the elements, element by element
    double *partials;        // per-block partial sums of the objective
};

// launchers (kernels_yz.hip, kernels_x.hip, kernels_util.hip, kernels_adj.hip) ------
hipError_t launch_ypass(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                        float2 *const *fields, int nfields, bool inverse,
                        const Counters *prologue, const SourceDev *src,
                        const SensorDev *sen = nullptr, float2 *const *dst = nullptr);
hipError_t launch_zfused(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                         int mode, float2 *const *in, float2 *const *out, float sa = 1.0f,
                         float sb = 1.0f, float2 *const *add0 = nullptr);
hipError_t launch_xvel(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, float2 *const *S, float *const *u,
                       const SourceDev &src, const SensorDev &sen, const Counters &cnt);
hipError_t launch_xden(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, const SourceDev &src, const SensorDev &sen,
                       const Counters &cnt, float2 *const *Sin, float *const *rho,
                       float *rho_total, float2 *const *Sout, bool rho0_sum_in_z = false,
                       float *const *rec = nullptr);
hipError_t launch_xeos(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, const SourceDev &src, const SensorDev &sen,
                       const Counters &cnt, float2 *const *Sin, const float *rho_total,
                       float2 *Sout, bool merged = false);
// real field -> packed x-spectrum (forward) or back, scaled by `scale`
hipError_t launch_xfwd(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const float *src, float2 *dst);
hipError_t launch_xinv(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const float2 *src, float *dst, float scale);
// reverse-mode step pieces (kernels_adj.hip)
hipError_t launch_adj_weights(hipStream_t s, const GridDev &g, const Medium &m, float *w,
                              float scale);
// drive terms of the source points (before the den pass) and the per-element
// sums of their shares into dJ/ds_e(n) (after it)
hipError_t launch_adj_src(hipStream_t s, const AdjDev &a, const SourceDev &src, int n);
hipError_t launch_adj_src_sum(hipStream_t s, const AdjDev &a, int n);
// fused x-row passes of the reverse step (kw_adjx_*): p_spec and loss for the
// eos and lossless den passes; Sin / Sout the spectra they read and write
enum { ADJX_EOS = 0, ADJX_DEN = 1, ADJX_DEN_ABS = 2, ADJX_VEL = 3, ADJX_SUM = 4 };
hipError_t launch_adjx(hipStream_t s, int pass, const GridDev &g, const LaunchCfg &c,
                       const Tables &t, const Medium &m, const SourceDev &src, const AdjDev &ad,
                       const float2 *p_spec, bool loss, float2 *const *Sin, float2 *const *Sout);
// objective J into *out through per-block partials (adj_objective_blocks of them)
int adj_objective_blocks(const GridDev &g);
hipError_t launch_adj_objective(hipStream_t s, const GridDev &g, const float *w,
                                const float *sum2, double *partials, double *out);
// the static scratch array of kw_create_static (static_scratch.hip): its
// device address on the current device and its size
constexpr size_t kStaticScratchBytes = (size_t)96 << 20;
hipError_t static_scratch(void **out, size_t *bytes);
hipError_t launch_fill(hipStream_t s, float *p, size_t n, float v);
hipError_t launch_scale(hipStream_t s, const float *src, float *dst, size_t n, float scale);
hipError_t launch_fill_int(hipStream_t s, int *p, size_t n, int v);
// dst[i] = f(sum2[i]) for the gather of p_rms / intensity
hipError_t launch_finalize(hipStream_t s, const float *sum2, float *dst, size_t n, float inv_count,
                           int mode, Coef rho0, Coef c0sq, const int *index);

}  // namespace kw
