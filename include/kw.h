/*
 * kw.h -- C ABI of the MI355X (gfx950) k-space pseudospectral solver.
 *
 * One simulation advances the coupled first-order equations of
 * Jaros, Rendell & Treeby (Section 2.2): the spectral pressure gradient and
 * velocity update, Eqs. (4a)-(4b); the spectral velocity divergence and split
 * density update with the nonlinear denominator, Eqs. (4c)-(4d); the
 * equation of state with the B/A term, Eq. (6); and the power-law absorption
 * and dispersion terms through fractional Laplacians, Eq. (8).  Wavenumbers
 * follow Eq. (5); the k-space correction is kappa = sinc(c_ref k dt / 2).
 * The split-field PML (Section 2.2) is applied inside the grid.
 *
 * Every step runs on the GPU: 3D real-to-complex / complex-to-real FFTs made of
 * hand-written HIP passes, with the element-wise updates fused into them.
 * There is no host round trip inside kw_step.
 *
 * Conventions
 *   - Grid point (x, y, z) has the flat index x + nx*(y + ny*z) (x fastest).
 *   - Host arrays passed to kw_create / kw_set_field are copied before the call
 *     returns; the caller keeps ownership of them.
 *   - The device workspace is owned by the caller (typically a torch uint8
 *     tensor); the library borrows it from kw_create until kw_destroy and
 *     carves every device array out of it.  The library allocates no device
 *     memory of its own (kw_create and kw_gather use no hipMalloc).
 *   - All device work is enqueued on the stream given to kw_create
 *     (a hipStream_t passed as void*; NULL is the default stream).
 *   - Every function returns a status code; on failure kw_last_error() gives a
 *     thread-local message.  Nothing aborts and no exception crosses the ABI.
 *   - Threads: kw_prepare, kw_plan_workspace_size and kw_plan_destroy make no
 *     HIP call and may run in any number of host threads at once.  Every
 *     other call may use the device; make all of them from one host thread.
 *     Several simulations may be driven from that thread, each on a stream of
 *     its own, and their work then overlaps on the GPU.  Simulations that share
 *     a stream are serialised on it.  Device calls from several host threads
 *     at once are not supported.
 */
#ifndef KW_H
#define KW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define KW_OK            0
#define KW_EINVAL       -1   /* bad argument, NULL pointer, out-of-range value          */
#define KW_EUNSUPPORTED -2   /* a dimension is not 2^a 3^b 5^c, too small/large, odd nx */
#define KW_ENOMEM       -3   /* workspace smaller than kw_workspace_size()              */
#define KW_EDEVICE      -4   /* HIP error (no device, launch failure, ...)              */
#define KW_ESTATE       -5   /* call not valid in the current state                     */
#define KW_ENONFINITE   -6   /* a NaN or Inf appeared in the pressure (see kw_stats)     */

/* medium flags */
#define KW_NONLINEAR     1u  /* B/A term of Eq. (6) and denominator of Eq. (4d)        */
#define KW_ABSORBING     2u  /* absorption and dispersion term L_d, Eq. (8)             */

/* recorded quantities (kw_sensor.record) and gather targets (kw_gather.what) */
#define KW_REC_P_MAX     1u  /* running maximum of p over recorded steps               */
#define KW_REC_P_RMS     2u  /* sqrt(mean p^2) over recorded steps                     */
#define KW_REC_P_SERIES  4u  /* p at the sensor points, one row per recorded step      */
#define KW_REC_P_FINAL   8u  /* p on the whole grid after the last step                */
#define KW_REC_U_FINAL  16u  /* ux, uy, uz (staggered) after the last step, 3 fields   */
#define KW_REC_INTENSITY 32u /* time-mean p^2 / (rho0 c0) at the sensor points         */
#define KW_REC_P_MIN     64u /* running minimum of p (peak negative pressure)          */
#define KW_REC_HARMONICS 128u /* complex amplitudes of harmonics 1..n_harmonics of
                                harmonic_freq: A_h = (2/N) sum_m p^m e^{-i h 2 pi f m dt}
                                over the N recorded steps m, per sensor point          */
#define KW_REC_U_SERIES  256u /* u_x, u_y, u_z (staggered) at the sensor points, one
                                row of 3 x points per recorded step (mask sensor only) */

/* fields for kw_set_field / kw_gather_field (whole grid, float32) */
#define KW_FIELD_P       1   /* acoustic pressure p^n                                  */
#define KW_FIELD_UX      2   /* particle velocity u_x^(n-1/2) at x + dx/2              */
#define KW_FIELD_UY      3
#define KW_FIELD_UZ      4
#define KW_FIELD_RHOX    5   /* split acoustic density rho_x^n                          */
#define KW_FIELD_RHOY    6
#define KW_FIELD_RHOZ    7

typedef struct kw_sim kw_sim;

typedef struct kw_grid {
    int32_t nx, ny, nz;       /* points; nx even; every size of the form 2^a 3^b 5^c,
                                 4 <= n <= 1024 (nx <= 2048)                          */
    double  dx, dy, dz;       /* spacing [m], > 0                                       */
    double  dt;               /* time step [s]; 0 -> cfl * min(dx,dy,dz) / max(c0)     */
    double  cfl;              /* used when dt == 0                                      */
    int32_t pml_size[3];      /* PML points per side along x, y, z (inside the grid)   */
    double  pml_alpha[3];     /* PML strength [Np per grid point]                      */
} kw_grid;

/* Each property is either a host array of nx*ny*nz floats or, when the
 * pointer is NULL, the scalar next to it.  alpha0 is the power-law prefactor
 * in dB / (MHz^y cm), converted internally to Np (rad/s)^-y m^-1 as stated
 * with Eq. (3).  tau and eta follow Eq. (3). */
typedef struct kw_medium {
    const float *c0;      double c0_scalar;       /* sound speed [m/s]            */
    const float *rho0;    double rho0_scalar;     /* ambient density [kg/m^3]     */
    const float *alpha0;  double alpha0_scalar;   /* dB / (MHz^y cm)              */
    const float *bona;    double bona_scalar;     /* nonlinearity parameter B/A   */
    double   alpha_power;                         /* y, 0 < y < 3, y != 1         */
    double   c_ref;                               /* kappa reference; 0 -> max c0 */
    uint32_t flags;                               /* KW_NONLINEAR | KW_ABSORBING  */
} kw_medium;

/* Source kinds (the source enters the model through the mass source term of
 * Eq. (4d) or the force term of Eq. (4b); Section 3.4 describes injection as
 * updating the pressure or the particle velocity at the source points):
 *   KW_SOURCE_MASS      s_e [Pa] as an additive mass source split evenly over
 *                       the three density components, M_xi = 2 s / (3 c0 dx),
 *                       added after the update of Eq. (4d), at t = (n + 1/2) dt;
 *   KW_SOURCE_FORCE     s_e [m/s^2] as an additive force per unit mass F on
 *                       the velocity component `axis`, u += dt F after the
 *                       update of Eq. (4b), at t = n dt;
 *   KW_SOURCE_PRESSURE  Dirichlet: p^(n+1) = s_e [Pa] at the points after the
 *                       equation of state, at t = (n + 1) dt (the densities
 *                       are not changed). */
#define KW_SOURCE_MASS      0
#define KW_SOURCE_FORCE     1
#define KW_SOURCE_PRESSURE  2

/* Drive s_e(t) of each element at the listed grid points:
 * s_e = amp[e] sin(2 pi freq t + phase[e]) with t as stated for the kind, or
 * signal[e * n_samples + n] in step n when signal is non-NULL (0 after the
 * last sample). */
typedef struct kw_source {
    int64_t        n_points;     /* 0 -> no source                                 */
    const int64_t *index;        /* flat indices, strictly increasing               */
    const int32_t *element;      /* element of each point; NULL -> all element 0   */
    int32_t        n_elements;   /* >= 1 when n_points > 0                          */
    const float   *amp;          /* [n_elements] (unit of the kind)                 */
    const float   *phase;        /* [n_elements] rad                                */
    double         freq;         /* Hz                                              */
    const float   *signal;       /* optional [n_elements * n_samples]               */
    int32_t        n_samples;
    int32_t        kind;         /* KW_SOURCE_*                                     */
    int32_t        axis;         /* KW_SOURCE_FORCE: 0 = x, 1 = y, 2 = z            */
} kw_source;

/* Sensor: quantities in `record` are kept for the points in `index` (strictly
 * increasing) or for every grid point when index == NULL (n_points ignored).
 * The pressure p^(n) after step n is recorded when n >= record_start (>= 1),
 * and with it u^(n-1/2) for KW_REC_U_SERIES.  The paper's application keeps
 * peak positive and negative pressure over the domain and the time-varying
 * pressure and velocity over a region (Section 5); the harmonic amplitudes are
 * an on-device reduction of that time series. */
typedef struct kw_sensor {
    uint32_t       record;
    int64_t        n_points;
    const int64_t *index;
    int32_t        record_start;
    int32_t        series_capacity;   /* rows kept for KW_REC_P_SERIES / KW_REC_U_SERIES */
    int32_t        n_harmonics;       /* 1..16 with KW_REC_HARMONICS                       */
    double         harmonic_freq;     /* [Hz]; 0 -> the source frequency                  */
} kw_sensor;

typedef struct kw_stats_t {
    int64_t steps;             /* steps taken                                        */
    int64_t nonfinite_step;    /* first step with a NaN/Inf pressure, -1 if none     */
    double  dt;                /* time step used [s]                                  */
    double  c_ref;             /* reference sound speed used [m/s]                    */
    int64_t workspace_bytes;   /* bytes of the workspace actually used                */
    int32_t fft_forward_per_step;  /* 3D forward transforms per step (Section 3.4)   */
    int32_t fft_inverse_per_step;  /* 3D inverse transforms per step                  */
    int32_t kernels_per_step;      /* kernel launches per step                        */
    int32_t n_classes;             /* kernel classes with timing below                */
    char    class_name[16][24];    /* kernel class names                              */
    double  class_ms[16];          /* summed device time per class (profiling on)     */
    int64_t class_launches[16];    /* launches per class while profiling              */
    double  class_bytes[16];       /* mean algorithmic HBM bytes per launch of the class */
} kw_stats_t;

/* Device bytes needed by a simulation with these inputs (the same number is
 * the admission footprint of the serving layer).  0 when the inputs are
 * invalid (kw_last_error says why). */
size_t kw_workspace_size(const kw_grid *grid, const kw_medium *medium,
                         const kw_source *source, const kw_sensor *sensor);

/* Validate the inputs (before any device call), precompute the 1D operator
 * tables and per-point medium coefficients in float64 on the host, carve the
 * workspace, upload, and zero the state (p = u = rho = 0).  `source` and
 * `sensor` may be NULL.  On success *out owns host-side state only. */
int kw_create(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
              const kw_sensor *sensor, void *dev_workspace, size_t ws_bytes,
              void *stream, kw_sim **out);

/* Set-up in two parts, for callers that prepare simulations off the thread
 * that drives the GPU (a serving loop):
 *   kw_prepare       everything kw_create does on the host -- validation, FFT
 *                    plans, the 1D operator tables of Eqs. (4a), (4c), (5), (8)
 *                    and the per-point medium coefficients in float64, source
 *                    and sensor lists -- and no HIP call.  The host arrays of
 *                    the inputs are copied; *out owns host memory only.  Same
 *                    status codes as kw_create for invalid inputs.
 *   kw_plan_workspace_size  device bytes kw_create_prepared needs (equal to
 *                    kw_workspace_size of the same inputs); 0 for NULL.
 *   kw_create_prepared  the device part of kw_create: binds a workspace and a
 *                    stream, uploads and zeroes the state (KW_EINVAL for a NULL
 *                    or misaligned workspace, KW_ENOMEM when it is too small,
 *                    KW_EDEVICE for a HIP error).  The plan is only read: it may
 *                    be destroyed afterwards or used for more simulations.
 *   kw_plan_destroy  frees the plan; NULL-safe.
 * kw_create is kw_prepare followed by kw_create_prepared. */
typedef struct kw_plan kw_plan;
int kw_prepare(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
               const kw_sensor *sensor, kw_plan **out);
size_t kw_plan_workspace_size(const kw_plan *plan);
int kw_create_prepared(const kw_plan *plan, void *dev_workspace, size_t ws_bytes, void *stream,
                       kw_sim **out);
int kw_plan_destroy(kw_plan *plan);

/* For callers that cannot allocate device memory beyond their inputs and
 * outputs (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): kw_create with the six spectral scratch arrays of the
 * step (packed half spectra, dead between steps) taken from one static array
 * of the library instead of the workspace.  The workspace then needs
 *     kw_workspace_size(...) - 6 S bytes,   S = 256 * ceil(4 * nx * ny * nz / 256),
 * and the six arrays must fit the static array of 96 MiB (6 S <= 100663296
 * bytes: grids up to about 4.19 million points, 160^3 for instance); larger
 * grids fail with KW_EUNSUPPORTED before any device work.  Neither this call
 * nor any later call on the simulation allocates device memory.  Every
 * simulation made this way on one GPU shares that GPU's array, which keeps
 * the last call's contents (nothing needs clearing: a step writes the arrays
 * before reading them): their steps, gathers and reverse steps must not
 * overlap in time, or they race.  Other statuses as kw_create. */
int kw_create_static(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
                     const kw_sensor *sensor, void *dev_workspace, size_t ws_bytes, void *stream,
                     kw_sim **out);

/* Enqueue n >= 0 time steps on the simulation's stream and return. */
int kw_step(kw_sim *sim, int32_t n);

/* Copy a recorded quantity (one KW_REC_* bit) into dst, as float32:
 *   P_MAX, P_MIN, P_RMS, INTENSITY: one value per sensor point (or grid point);
 *   P_SERIES: rows x sensor points, rows = min(recorded steps, capacity);
 *   U_SERIES: rows x 3 x sensor points;
 *   HARMONICS: n_harmonics x points x 2 (real, imaginary);
 *   P_FINAL: nx*ny*nz values; U_FINAL: 3*nx*ny*nz values (ux, uy, uz).
 * dst is device memory when dst_is_device != 0, else host memory.  The call
 * synchronizes the stream; it fails with KW_EINVAL when dst_bytes is too
 * small (the needed size is reported by kw_gather_bytes) and returns
 * KW_ENONFINITE (after copying) when a NaN/Inf pressure was detected. */
int kw_gather(kw_sim *sim, uint32_t what, void *dst, size_t dst_bytes, int dst_is_device);
int64_t kw_gather_bytes(kw_sim *sim, uint32_t what);

/* Overwrite one state field (KW_FIELD_*) with nx*ny*nz float32 values from
 * host (src_is_device == 0) or device memory.  Setting the pressure does not
 * touch the density components; initial-value problems set both. */
int kw_set_field(kw_sim *sim, int field, const void *src, int src_is_device);
/* Read one state field (KW_FIELD_*) into dst (nx*ny*nz float32).  The
 * pressure is transformed back from its spectrum through kw_gather, whose
 * status is returned unchanged. */
int kw_gather_field(kw_sim *sim, int field, void *dst, int dst_is_device);

/* Per-kernel-class device timing with HIP events around every launch on the
 * simulation's stream (off by default; launches are eager while it is on). */
int kw_profile(kw_sim *sim, int on);
int kw_stats(kw_sim *sim, kw_stats_t *out);

/* Use captured HIP graphs of `steps_per_graph` steps for kw_step (0 = off,
 * the default is 8). */
int kw_set_graph(kw_sim *sim, int32_t steps_per_graph);

/* Override the FFT radix schedule of one axis (0 = x, 1 = y, 2 = z) and its
 * tile: columns per block of the y/z passes, rows per block of the x passes
 * (0 = the default).  radices lists the factors of the transform length in
 * forward order (product must equal the length: nx/2 for x).  For a
 * power-of-two length, radices of at most 4, 8 or 16 (each a power of two)
 * run on the 4-, 8- or 16-wide fixed engine, and a schedule of radix-32
 * passes only on the 32-wide one; for a length with a factor 3 or 5, radices
 * that all divide 12 or 20 on the 12- or 20-wide fixed engine; other
 * schedules on the generic one.  Used by the autotuner; must be called
 * before the first kw_step.
 * Returns KW_EINVAL for radices that do not form a schedule of the length,
 * KW_EUNSUPPORTED for a tile that does not fit a block (the plan is then
 * left as it was), KW_ESTATE after the first step. */
int kw_set_plan(kw_sim *sim, int axis, const int32_t *radices, int32_t n_radices,
                int32_t tile);

/* State snapshots (checkpoint / restart, Section 3.4: a run can be stopped
 * and resumed from its saved state).  A snapshot holds the step counter, the
 * non-finite flag, u_x, u_y, u_z, rho_x, rho_y, rho_z, the pressure (as its
 * packed spectrum) and the sensor accumulators, behind a header that records
 * the set-up it belongs to.  kw_state_bytes gives its size (-1 for NULL).
 * kw_save writes it to dst (device memory when dst_is_device != 0, else host
 * memory); kw_load restores it into a simulation created with the same grid,
 * medium flags, time step and sensor set-up (KW_EINVAL otherwise, before
 * anything is overwritten).  Continuing after kw_load gives bit-for-bit the
 * results of the run that was saved.  Both calls synchronize the stream. */
int64_t kw_state_bytes(kw_sim *sim);
int kw_save(kw_sim *sim, void *dst, size_t dst_bytes, int dst_is_device);
int kw_load(kw_sim *sim, const void *src, size_t src_bytes, int src_is_device);

/* Reverse mode: the discrete adjoint of kw_step for the objective
 *   J = sum_x w(x) I(x),  I(x) = (1/N_w) sum_m p^m(x)^2 / (rho0 c0)(x),
 * the time-mean intensity over the recorded steps m = record_start..n_steps
 * (sensor.record_start of the simulation; the intensity output of Section 5),
 * differentiated with respect to the drive values s_e(n) of the source
 * elements and, for a sinusoidal drive, their amplitudes and phases.  Each
 * reverse step applies the transpose of one forward step, Eqs. (4a)-(4d), (6),
 * (8), in float32 on the GPU, using the forward state after that step.
 *
 *   kw_adjoint_workspace_size  device bytes for n_steps forward steps (0 on error)
 *   kw_adjoint_create  weights: host array of nx*ny*nz floats w(x); the adjoint
 *                      borrows the caller-owned device workspace, uses the
 *                      simulation's stream and spectral scratch, and keeps a
 *                      pointer to `sim` (which must outlive it).  The source
 *                      must be set (KW_EINVAL otherwise).
 *   kw_adjoint_step    reverse step n: `sim` must hold the state after forward
 *                      step n (for example restored with kw_load), else
 *                      KW_ESTATE; call it for n = n_steps-1 down to 0.  Between
 *                      reverse steps the simulation may be stepped or loaded
 *                      freely (the adjoint state lives in its own workspace).
 *   kw_adjoint_record  advances `sim` by one step, as kw_step(sim, 1) does
 *                      (launched without the step graph), and writes to
 *                      dev_record (device memory, kw_adjoint_record_bytes)
 *                      what the reverse step needs of it: du_x, du_y, du_z of
 *                      Eq. (4c), rho_x, rho_y, rho_z after Eq. (4d) and the
 *                      packed spectrum of the new pressure.  KW_EINVAL for a
 *                      short buffer.  Asynchronous on the simulation's stream.
 *   kw_adjoint_step_record  reverse step n reading the forward state from a
 *                      record of forward step n made by kw_adjoint_record
 *                      (the caller keeps each record with its step); `sim`
 *                      may hold any state.  Without recomputing du_xi and
 *                      without restoring a snapshot, it is the cheaper way to
 *                      run a checkpointed sweep: restore a checkpoint, record
 *                      the steps up to the next one, reverse them.
 *   kw_adjoint_objective  J of the forward run, once `sim` holds the state after
 *                      its last step n_steps - 1 (needs p_rms or intensity
 *                      recorded at every point); float64 sum on the device
 *   kw_adjoint_source_gradient  dJ/ds_e(n) as double [n_steps][n_elements] (host)
 *   kw_adjoint_gradient  dJ/da_e and dJ/dphi_e (host, n_elements each); needs a
 *                      sinusoidal drive (KW_EINVAL for a sampled signal)
 *   kw_adjoint_destroy frees host state only; NULL-safe. */
typedef struct kw_adj kw_adj;
size_t kw_adjoint_workspace_size(kw_sim *sim, int32_t n_steps);
int kw_adjoint_create(kw_sim *sim, const float *weights, int32_t n_steps, void *dev_workspace,
                      size_t ws_bytes, kw_adj **out);
int kw_adjoint_objective(kw_adj *adj, double *J);
int kw_adjoint_step(kw_adj *adj, int32_t n);
int64_t kw_adjoint_record_bytes(kw_adj *adj);
int kw_adjoint_record(kw_adj *adj, void *dev_record, size_t bytes);
int kw_adjoint_step_record(kw_adj *adj, int32_t n, const void *dev_record, size_t bytes);
int kw_adjoint_source_gradient(kw_adj *adj, double *dJds, size_t dst_bytes);
int kw_adjoint_gradient(kw_adj *adj, double *grad_amp, double *grad_phase);
int kw_adjoint_destroy(kw_adj *adj);

/* Free library-owned host state (never the workspace).  NULL-safe. */
int kw_destroy(kw_sim *sim);

/* Thread-local message describing the last failure. */
const char *kw_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KW_H */
