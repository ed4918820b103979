// Host side of the C ABI declared in include/kw.h: validation, float64
// precomputation of the 1D operator tables and per-point medium coefficients,
// workspace carving, the per-step launch sequence, HIP graphs and profiling.
#include "kw.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kw_internal.h"

using namespace kw;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define KW_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(KW_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;

bool smooth235(long n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// ---------------------------------------------------------------------------
// FFT radix schedules
// ---------------------------------------------------------------------------
const int kRadices16[] = {16, 15, 12, 10, 8, 6, 5, 4, 3, 2};
const int kRadices32[] = {32, 30, 25, 24, 20, 16, 15, 12, 10, 8, 6, 5, 4, 3, 2};

void search(int n, int maxr, std::vector<int> &cur, std::vector<int> &best, int &best_np,
            int &best_min) {
    if (n == 1) {
        const int np = (int)cur.size();
        const int mn = cur.empty() ? 1 : *std::min_element(cur.begin(), cur.end());
        if (np < best_np || (np == best_np && mn > best_min)) {
            best = cur;
            best_np = np;
            best_min = mn;
        }
        return;
    }
    if ((int)cur.size() >= kMaxPasses) return;
    const int *rs = (maxr > 16) ? kRadices32 : kRadices16;
    const int nr = (maxr > 16) ? (int)(sizeof kRadices32 / sizeof(int))
                               : (int)(sizeof kRadices16 / sizeof(int));
    for (int i = 0; i < nr; ++i) {
        const int r = rs[i];
        if (r > maxr || n % r) continue;
        if (!cur.empty() && r > cur.back()) continue;  // non-increasing: no duplicates
        cur.push_back(r);
        search(n / r, maxr, cur, best, best_np, best_min);
        cur.pop_back();
    }
}

bool plan_from_radices(int n, const std::vector<int> &rad, FftPlan &p) {
    if (rad.empty() || (int)rad.size() > kMaxPasses) return false;
    long prod = 1;
    p = FftPlan{};
    p.n = n;
    p.np = (int)rad.size();
    p.L = 0;
    p.rmax = 0;
    for (int i = 0; i < p.np; ++i) {
        const int r = rad[i];
        bool okr = false;
        for (int q : kRadices32) okr |= (q == r);
        if (!okr) return false;
        p.radix[i] = r;
        p.code |= (unsigned long long)r << (6 * i);
        prod *= r;
        p.L = std::max(p.L, n / r);
        p.rmax = std::max(p.rmax, r);
    }
    return prod == n;
}

bool generic_plan(int n, FftPlan &p) {
    if (n < 2) return false;
    std::vector<int> cur, best;
    int best_np = INT_MAX, best_min = 0;
    search(n, 16, cur, best, best_np, best_min);
    // fall back to radices up to 32 when that saves a pass
    std::vector<int> best32;
    int np32 = INT_MAX, min32 = 0;
    cur.clear();
    search(n, 32, cur, best32, np32, min32);
    if (np32 < best_np) {
        best = best32;
        best_np = np32;
    }
    if (best.empty()) return false;
    std::sort(best.begin(), best.end());   // smaller radices first
    return plan_from_radices(n, best, p);
}

FftPlan reversed(const FftPlan &p) {
    FftPlan q = p;
    q.code = 0;
    for (int i = 0; i < p.np; ++i) {
        q.radix[i] = p.radix[p.np - 1 - i];
        q.code |= (unsigned long long)q.radix[i] << (6 * i);
    }
    return q;
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Default elements per thread of the fixed-width engine for a power-of-two
// length: 16 for the column passes, 8 for the x rows (whose fused updates keep
// more values live); short transforms use 8.
int fixed_width(int n, int axis) { return (axis > 0 && n >= 64) ? 16 : 8; }

bool fixed_plan_from_radices(int n, int E, const std::vector<int> &rad, FftPlan &p) {
    if (rad.empty() || (int)rad.size() > kMaxPasses) return false;
    long prod = 1;
    p = FftPlan{};
    p.n = n;
    p.np = (int)rad.size();
    p.L = n / E;
    p.rmax = 0;
    for (int i = 0; i < p.np; ++i) {
        const int r = rad[i];
        // (the 32-wide engine runs radix-32 passes only)
        if (r < 2 || r > E || E % r || (E == 32 && r != 32)) return false;
        p.radix[i] = r;
        p.code |= (unsigned long long)r << (6 * i);
        prod *= r;
        p.rmax = std::max(p.rmax, r);
    }
    return prod == n && n % E == 0;
}

// Width of the mixed-radix fixed engine for a length with a factor 3 (E = 12)
// and a default schedule: radices dividing E, largest first (0 when the
// length has no such schedule, e.g. a factor 9).  Lengths with a factor 5 stay
// on the generic engine unless a caller schedule asks for E = 20: measured on
// the 160^3 grid, every axis ran 2-6 % faster on the generic engine (the
// 20-wide engine holds 40 registers of data per thread), while the 12-wide
// engine made the 192^3 step 13 % faster.
int mixed_width(int n, std::vector<int> &r) {
    for (int E : {12}) {
        if (n % E) continue;
        std::vector<int> divs;
        for (int q = E; q >= 2; --q)
            if (E % q == 0) divs.push_back(q);
        r.clear();
        int m = n;
        while (m > 1) {
            int q = 0;
            for (int d : divs)
                if (m % d == 0) { q = d; break; }
            if (q == 0) break;
            r.push_back(q);
            m /= q;
        }
        if (m == 1 && (int)r.size() <= kMaxPasses) return E;
    }
    r.clear();
    return 0;
}

// Choose the engine and plans of one axis of transform length n.  `rad`, when
// given, is a caller-chosen radix schedule (the autotuner's).
bool axis_plan(int n, int axis, const std::vector<int> *rad, int &eng, FftPlan &f, FftPlan &i) {
    if (!is_pow2(n) && n >= 24) {
        // lengths 2^a 3 and 2^a 5: the fixed engine at width 12 or 20; a caller
        // schedule runs there when all its radices divide one of the widths
        std::vector<int> r;
        int E = 0;
        if (rad) {
            for (int w : {12, 20}) {
                bool all = n % w == 0;
                for (int q : *rad) all = all && w % q == 0;
                if (all) { E = w; break; }
            }
            r = *rad;
        } else {
            E = mixed_width(n, r);
        }
        if (E && fixed_plan_from_radices(n, E, r, f)) {
            eng = E == 12 ? ENG_F12 : ENG_F20;
            // a plan of radices 6 and 4 runs on the kernels built for them
            if (E == 12 && std::all_of(r.begin(), r.end(), [](int q) { return q == 6 || q == 4; }))
                eng = ENG_F12_64;
            i = f;
            return true;
        }
    }
    if (is_pow2(n) && n >= 16) {
        int E = fixed_width(n, axis);
        std::vector<int> r;
        if (rad) {
            r = *rad;
            // the width is the largest radix of a caller-chosen schedule (a
            // schedule with radix 32 and smaller radices is not a fixed-engine
            // plan: it runs on the generic engine)
            const int rm = *std::max_element(r.begin(), r.end());
            E = rm > 16 ? 32 : rm > 8 ? 16 : rm > 4 ? 8 : 4;
        } else {
            int m = n;
            while (m > 1) {
                int q = E;
                while (m % q) q /= 2;
                r.push_back(q);
                m /= q;
            }
        }
        if (fixed_plan_from_radices(n, E, r, f)) {
            eng = E == 32 ? ENG_F32 : E == 16 ? ENG_F16 : E == 8 ? ENG_F8 : ENG_F4;
            // plans of radix-E passes only, and 8-wide plans of radices 8
            // and 4, run on the kernels built for those radices
            if ((E == 8 || E == 16) && std::all_of(r.begin(), r.end(), [E](int q) { return q == E; }))
                eng = E == 16 ? ENG_F16P : ENG_F8P;
            else if (E == 8 && std::all_of(r.begin(), r.end(), [](int q) { return q == 8 || q == 4; }))
                eng = ENG_F8_84;
            i = f;
            return true;
        }
        if (!rad) return false;
        // a caller schedule outside the fixed engine's radices runs on the generic one
    }
    if (rad) {
        if (!plan_from_radices(n, *rad, f)) return false;
    } else if (!generic_plan(n, f)) {
        return false;
    }
    eng = f.rmax > 16 ? ENG_G32 : ENG_G16;
    i = reversed(f);
    return true;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + kAlign - 1) / kAlign * kAlign;
        return o;
    }
};

struct Layout {
    size_t counters, drive;
    size_t tw_x, tw_post, tw_y, tw_z, kx, ky, kz, dpx, dmx, dpy, dmy, dpz, dmz;
    size_t pml[6];
    size_t src_row, src_x, src_e, src_c, src_ac, src_as, src_sig;
    size_t sen_row, sen_x, sen_id, sen_idx, p_max, p_sum2, series, p_min, harm, hw, useries;
    size_t med[8];             // dtr x, y, z, rho0, c0sq, nl, ta, tb
    size_t u[3], rho[3], rho_total;
    size_t S[7];
    size_t total;
};

enum { MED_DTRX = 0, MED_DTRY, MED_DTRZ, MED_RHO0, MED_C0SQ, MED_NL, MED_TA, MED_TB };

// Which derived per-point maps are needed (true) or scalars (false).
struct MediumShape {
    bool het[8];
};

MediumShape medium_shape(const kw_medium *m) {
    MediumShape s{};
    const bool c = m->c0 != nullptr, r = m->rho0 != nullptr, a = m->alpha0 != nullptr,
               b = m->bona != nullptr;
    s.het[MED_DTRX] = s.het[MED_DTRY] = s.het[MED_DTRZ] = r;
    s.het[MED_RHO0] = r;
    s.het[MED_C0SQ] = c;
    s.het[MED_NL] = (m->flags & KW_NONLINEAR) && (c || r || b);
    s.het[MED_TA] = s.het[MED_TB] = (m->flags & KW_ABSORBING) && (c || a);
    return s;
}

struct Counts {
    long n_src = 0, n_sen = 0;
    bool sen_all = false;
    int n_elem = 0, n_samples = 0;
    uint32_t record = 0;
    int capacity = 0;
    int n_harm = 0;
    double harm_freq = 0.0;
};

Layout make_layout(const kw_grid *g, const kw_medium *m, const Counts &c) {
    Layout L{};
    Carver cv;
    const size_t nx = g->nx, ny = g->ny, nz = g->nz;
    const size_t N = nx * ny * nz, M = nx / 2, rows = ny * nz;
    L.counters = cv.take(2 * sizeof(int));
    L.drive = cv.take(std::max(1, c.n_elem) * sizeof(float));
    L.tw_x = cv.take(M * sizeof(float2));
    L.tw_post = cv.take(M * sizeof(float2));
    L.tw_y = cv.take(ny * sizeof(float2));
    L.tw_z = cv.take(nz * sizeof(float2));
    L.kx = cv.take((M + 1) * sizeof(float));
    L.ky = cv.take(ny * sizeof(float));
    L.kz = cv.take(nz * sizeof(float));
    L.dpx = cv.take((M + 1) * sizeof(float2));
    L.dmx = cv.take((M + 1) * sizeof(float2));
    L.dpy = cv.take(ny * sizeof(float2));
    L.dmy = cv.take(ny * sizeof(float2));
    L.dpz = cv.take(nz * sizeof(float2));
    L.dmz = cv.take(nz * sizeof(float2));
    L.pml[0] = cv.take(nx * sizeof(float));
    L.pml[1] = cv.take(nx * sizeof(float));
    L.pml[2] = cv.take(ny * sizeof(float));
    L.pml[3] = cv.take(ny * sizeof(float));
    L.pml[4] = cv.take(nz * sizeof(float));
    L.pml[5] = cv.take(nz * sizeof(float));
    if (c.n_src > 0) {
        L.src_row = cv.take((rows + 1) * sizeof(int));
        L.src_x = cv.take(c.n_src * sizeof(int));
        L.src_e = cv.take(c.n_src * sizeof(int));
        L.src_c = cv.take(c.n_src * sizeof(float));
        L.src_ac = cv.take(c.n_elem * sizeof(double));
        L.src_as = cv.take(c.n_elem * sizeof(double));
        if (c.n_samples > 0) L.src_sig = cv.take((size_t)c.n_elem * c.n_samples * sizeof(float));
    }
    const size_t nrec = c.sen_all ? N : (size_t)c.n_sen;
    if (!c.sen_all && c.n_sen > 0) {
        L.sen_row = cv.take((rows + 1) * sizeof(int));
        L.sen_x = cv.take(c.n_sen * sizeof(int));
        L.sen_id = cv.take(c.n_sen * sizeof(int));
        L.sen_idx = cv.take(c.n_sen * sizeof(int));
    }
    if (nrec > 0 && (c.record & KW_REC_P_MAX)) L.p_max = cv.take(nrec * sizeof(float));
    if (nrec > 0 && (c.record & (KW_REC_P_RMS | KW_REC_INTENSITY)))
        L.p_sum2 = cv.take(nrec * sizeof(float));
    if (!c.sen_all && c.n_sen > 0 && (c.record & KW_REC_P_SERIES) && c.capacity > 0)
        L.series = cv.take((size_t)c.capacity * c.n_sen * sizeof(float));
    if (nrec > 0 && (c.record & KW_REC_P_MIN)) L.p_min = cv.take(nrec * sizeof(float));
    if (nrec > 0 && (c.record & KW_REC_HARMONICS)) {
        L.harm = cv.take((size_t)2 * c.n_harm * nrec * sizeof(float));
        L.hw = cv.take((size_t)2 * c.n_harm * sizeof(float));
    }
    if (!c.sen_all && c.n_sen > 0 && (c.record & KW_REC_U_SERIES) && c.capacity > 0)
        L.useries = cv.take((size_t)c.capacity * 3 * c.n_sen * sizeof(float));
    const MediumShape ms = medium_shape(m);
    for (int i = 0; i < 8; ++i)
        if (ms.het[i]) L.med[i] = cv.take(N * sizeof(float));
    for (int i = 0; i < 3; ++i) L.u[i] = cv.take(N * sizeof(float));
    for (int i = 0; i < 3; ++i) L.rho[i] = cv.take(N * sizeof(float));
    if (m->flags & KW_ABSORBING) L.rho_total = cv.take(N * sizeof(float));
    for (int i = 0; i < 7; ++i) L.S[i] = cv.take(N * sizeof(float));
    L.total = cv.off;
    return L;
}

// ---------------------------------------------------------------------------
// validation (no device calls)
// ---------------------------------------------------------------------------
int validate(const kw_grid *g, const kw_medium *m, const kw_source *s, const kw_sensor *z,
             Counts &c) {
    if (!g || !m) return fail(KW_EINVAL, "grid and medium must not be NULL");
    const int dims[3] = {g->nx, g->ny, g->nz};
    const char *nm = "xyz";
    for (int a = 0; a < 3; ++a) {
        const int lim = (a == 0) ? 2048 : 1024;
        if (dims[a] < 4 || dims[a] > lim)
            return fail(KW_EUNSUPPORTED, "n%c = %d outside [4, %d]", nm[a], dims[a], lim);
        if (!smooth235(dims[a]))
            return fail(KW_EUNSUPPORTED, "n%c = %d is not of the form 2^a 3^b 5^c", nm[a], dims[a]);
    }
    if (g->nx % 2) return fail(KW_EUNSUPPORTED, "nx = %d must be even", g->nx);
    if ((long)g->nx * g->ny * g->nz >= (1L << 31))
        return fail(KW_EUNSUPPORTED, "grid has 2^31 or more points");
    const double sp[3] = {g->dx, g->dy, g->dz};
    for (int a = 0; a < 3; ++a) {
        if (!(sp[a] > 0.0) || !std::isfinite(sp[a]))
            return fail(KW_EINVAL, "spacing d%c must be positive", nm[a]);
        if (g->pml_size[a] < 0 || 2 * g->pml_size[a] > dims[a])
            return fail(KW_EINVAL, "pml_size[%d] = %d does not fit the grid", a, g->pml_size[a]);
        if (!(g->pml_alpha[a] >= 0.0)) return fail(KW_EINVAL, "pml_alpha must be >= 0");
    }
    if (g->dt < 0.0 || !std::isfinite(g->dt)) return fail(KW_EINVAL, "dt must be >= 0");
    if (g->dt == 0.0 && !(g->cfl > 0.0)) return fail(KW_EINVAL, "dt == 0 needs cfl > 0");
    if (m->flags & ~(KW_NONLINEAR | KW_ABSORBING)) return fail(KW_EINVAL, "unknown medium flags");
    if (!m->c0 && !(m->c0_scalar > 0.0)) return fail(KW_EINVAL, "c0 must be positive");
    if (!m->rho0 && !(m->rho0_scalar > 0.0)) return fail(KW_EINVAL, "rho0 must be positive");
    if (m->flags & KW_ABSORBING) {
        const double y = m->alpha_power;
        if (!(y > 0.0 && y < 3.0) || y == 1.0)
            return fail(KW_EINVAL, "alpha_power = %g: need 0 < y < 3 and y != 1", y);
        if (!m->alpha0 && !(m->alpha0_scalar >= 0.0)) return fail(KW_EINVAL, "alpha0 must be >= 0");
    }
    if (m->c_ref < 0.0) return fail(KW_EINVAL, "c_ref must be >= 0");
    const long N = (long)g->nx * g->ny * g->nz;
    c = Counts{};
    if (s && s->n_points > 0) {
        if (!s->index || !s->amp || !s->phase) return fail(KW_EINVAL, "source arrays missing");
        if (s->n_elements < 1) return fail(KW_EINVAL, "source n_elements must be >= 1");
        if (s->signal && s->n_samples < 1) return fail(KW_EINVAL, "signal needs n_samples >= 1");
        if (s->kind < KW_SOURCE_MASS || s->kind > KW_SOURCE_PRESSURE)
            return fail(KW_EINVAL, "unknown source kind %d", s->kind);
        if (s->kind == KW_SOURCE_FORCE && (s->axis < 0 || s->axis > 2))
            return fail(KW_EINVAL, "force source axis %d outside [0, 2]", s->axis);
        for (long i = 0; i < s->n_points; ++i) {
            if (s->index[i] < 0 || s->index[i] >= N)
                return fail(KW_EINVAL, "source index %ld out of the grid", (long)s->index[i]);
            if (i && s->index[i] <= s->index[i - 1])
                return fail(KW_EINVAL, "source indices must be strictly increasing");
            if (s->element && (s->element[i] < 0 || s->element[i] >= s->n_elements))
                return fail(KW_EINVAL, "source element id out of range");
        }
        c.n_src = s->n_points;
        c.n_elem = s->n_elements;
        c.n_samples = s->signal ? s->n_samples : 0;
    } else if (s && s->n_points < 0) {
        return fail(KW_EINVAL, "source n_points must be >= 0");
    }
    if (z) {
        if (z->record & ~511u) return fail(KW_EINVAL, "unknown record bits");
        if (z->record_start < 1) return fail(KW_EINVAL, "record_start must be >= 1");
        c.record = z->record;
        c.capacity = z->series_capacity;
        if (z->index) {
            if (z->n_points < 1) return fail(KW_EINVAL, "sensor n_points must be >= 1");
            for (long i = 0; i < z->n_points; ++i) {
                if (z->index[i] < 0 || z->index[i] >= N)
                    return fail(KW_EINVAL, "sensor index %ld out of the grid", (long)z->index[i]);
                if (i && z->index[i] <= z->index[i - 1])
                    return fail(KW_EINVAL, "sensor indices must be strictly increasing");
            }
            c.n_sen = z->n_points;
        } else {
            c.sen_all = true;
            if (z->record & KW_REC_P_SERIES)
                return fail(KW_EINVAL, "a pressure series needs a sensor index list");
        }
        if ((z->record & KW_REC_P_SERIES) && z->series_capacity < 1)
            return fail(KW_EINVAL, "a pressure series needs series_capacity >= 1");
        if (z->record & KW_REC_U_SERIES) {
            if (!z->index) return fail(KW_EINVAL, "a velocity series needs a sensor index list");
            if (z->series_capacity < 1)
                return fail(KW_EINVAL, "a velocity series needs series_capacity >= 1");
        }
        if (z->record & KW_REC_HARMONICS) {
            if (z->n_harmonics < 1 || z->n_harmonics > 16)
                return fail(KW_EINVAL, "n_harmonics = %d outside [1, 16]", z->n_harmonics);
            const double f = z->harmonic_freq > 0.0 ? z->harmonic_freq
                                                    : (s && s->n_points > 0 ? s->freq : 0.0);
            if (!(f > 0.0) || !std::isfinite(f))
                return fail(KW_EINVAL, "harmonics need harmonic_freq > 0 or a source frequency");
            c.n_harm = z->n_harmonics;
            c.harm_freq = f;
        }
    }
    return KW_OK;
}

// wavenumber of FFT index j on an axis of n points and spacing d (Eq. (5))
double wavenumber(int j, int n, double d) {
    const int m = (j <= (n - 1) / 2) ? j : j - n;
    return m * 2.0 * kPi / (d * n);
}

double pml_factor(int i, bool staggered, int n, int size, double alpha, double c_ref, double d,
                  double dt) {
    if (size <= 0 || alpha == 0.0) return 1.0;
    const double pos = i + (staggered ? 0.5 : 0.0);
    const double depth = std::max({size - pos, pos - (n - 1 - size), 0.0});
    const double sigma = alpha * (c_ref / d) * std::pow(depth / size, 4.0);
    return std::exp(-sigma * dt / 2.0);
}

}  // namespace

// ---------------------------------------------------------------------------
// the simulation object
// ---------------------------------------------------------------------------
struct kw_sim {
    kw_grid grid;
    uint32_t flags;
    hipStream_t stream;
    char *ws;
    size_t ws_used = 0;                // bytes of the workspace in use
    Layout L;
    Counts cnt;
    GridDev g;
    LaunchCfg cfg;
    Tables tab;
    Medium med;
    SourceDev src;
    SensorDev sen;
    Counters counters;
    StepBuffers buf;
    double dt, c_ref;
    int record_start;
    long steps = 0;
    bool stepped = false;
    // graphs
    int graph_steps = 8;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    // profiling
    bool profiling = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t max_lds = 64 * 1024;        // LDS bytes a block may use on this device
    bool merged_abs = false;           // absorption terms merged (scalar c0^2 tau, c0^2 eta)
    bool rho0_sum_in_z = false;        // absorbing with a constant rho0: the divergence
                                       // pass forms the spectrum of rho0 sum du
    float *rec[6] = {};                // while a step is recorded for the reverse mode:
                                       // where du_xi and the new rho_xi go (else null)
    // host copy of the source set-up (for the reverse-mode step)
    std::vector<int> src_flat, src_elem;
    std::vector<float> src_coef;
    std::vector<double> src_amp, src_phase;
    double class_ms[KC_COUNT] = {0};
    long class_n[KC_COUNT] = {0};
    double class_bytes[KC_COUNT] = {0};
    int kernels_per_step = 0;
    // per-launch algorithmic bytes
    double bytes[KC_COUNT] = {0};

    template <class T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

const char *kClassNames[KC_COUNT] = {"ypass_fwd", "ypass_inv", "zfused_grad", "zfused_div",
                                     "zfused_abs", "xvel",      "xden",        "xeos"};

hipEvent_t take_event(kw_sim *s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch one kernel (through `fn`), bracketed by events when profiling.
template <class F>
hipError_t launch_on(kw_sim *s, hipStream_t st, int cls, double nbytes, F fn) {
    if (!s->profiling) return fn();
    hipEvent_t a = take_event(s), b = take_event(s);
    if (!a || !b) return hipErrorOutOfMemory;
    (void)hipEventRecord(a, st);
    hipError_t e = fn();
    (void)hipEventRecord(b, st);
    s->recs.push_back({cls, a, b, nbytes});
    return e;
}
template <class F>
hipError_t launch(kw_sim *s, int cls, double nbytes, F fn) {
    return launch_on(s, s->stream, cls, nbytes, fn);
}

void resolve_profile(kw_sim *s) {
    if (s->recs.empty()) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto &r : s->recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            s->class_ms[r.cls] += ms;
            s->class_n[r.cls] += 1;
            s->class_bytes[r.cls] += r.bytes;
        }
        s->pool.push_back(r.a);
        s->pool.push_back(r.b);
    }
    s->recs.clear();
}

// Enqueue the kernels of one step.
hipError_t enqueue_step(kw_sim *s) {
    const GridDev &g = s->g;
    const LaunchCfg &c = s->cfg;
    const Tables &t = s->tab;
    hipStream_t st = s->stream;
    float2 *const *S = s->buf.S;
    const double unit = (double)g.nx * g.ny * g.nz * 4.0;
    const bool absorbing = s->med.absorbing;
    const MediumShape ms = [&] {
        MediumShape m{};
        m.het[MED_DTRX] = s->med.dtr[0].map != nullptr;
        m.het[MED_RHO0] = s->med.rho0.map != nullptr;
        m.het[MED_C0SQ] = s->med.c0sq.map != nullptr;
        m.het[MED_NL] = s->med.nl.map != nullptr;
        m.het[MED_TA] = s->med.ta.map != nullptr;
        return m;
    }();
    const double sens_units = (s->sen.all_points ? ((s->sen.p_max ? 2 : 0) + (s->sen.p_sum2 ? 2 : 0) +
                                                    (s->sen.p_min ? 2 : 0) +
                                                    (s->sen.harm ? 4 * s->sen.n_harm : 0))
                                                 : 0);
    hipError_t e;
    int nk = 0;
#define KW_L(cls, units, call)                                                  \
    do {                                                                        \
        e = launch(s, cls, (units) * unit, [&] { return (call); });             \
        if (e != hipSuccess) return e;                                          \
        ++nk;                                                                   \
    } while (0)

    float2 *s0[1] = {S[0]};
    float2 *s123[3] = {S[1], S[2], S[3]};
    float2 *s456[3] = {S[4], S[5], S[6]};
    float *const *rec = s->rec[0] ? s->rec : nullptr;
    KW_L(KC_YFWD, 2, launch_ypass(st, g, c, t, s0, 1, false, &s->counters, &s->src, &s->sen));
    KW_L(KC_ZGRAD, 4, launch_zfused(st, g, c, t, ZM_GRAD, s0, s123));
    KW_L(KC_YINV, 6, launch_ypass(st, g, c, t, s123, 3, true, nullptr, nullptr));
    KW_L(KC_XVEL, 12 + (ms.het[MED_DTRX] ? 3 : 0),
         launch_xvel(st, g, c, t, s->med, s123, s->buf.u, s->src, s->sen, s->counters));
    KW_L(KC_YFWD, 6, launch_ypass(st, g, c, t, s123, 3, false, nullptr, nullptr));
    if (s->rho0_sum_in_z) {
        // Constant rho0: the tau term of Eq. (8) transforms rho0 sum du, whose
        // (kx, ky) spectrum is rho0 nx ny times the sum of the three
        // divergence outputs of the z pass (S4..S6, before their y inverse
        // transform).  The y inverse transform writes them to S1..S3 instead
        // of in place, the density pass transforms rho alone (into S0), and
        // the absorption pass sums S4 + S5 + S6 as it loads its tau input: one
        // forward x and y transform less, and no write of a spectrum.
        const float r0nxny = (float)((double)s->med.rho0.scalar * g.nx * g.ny);
        KW_L(KC_ZDIV, 6, launch_zfused(st, g, c, t, ZM_DIV, s123, s456));
        KW_L(KC_YINV, 6, launch_ypass(st, g, c, t, s456, 3, true, nullptr, nullptr, nullptr, s123));
        float2 *rho_out[2] = {S[0], S[0]};
        KW_L(KC_XDEN, 11, launch_xden(st, g, c, t, s->med, s->src, s->sen, s->counters, s123,
                                      s->buf.rho, s->buf.rho_total, rho_out, true, rec));
        KW_L(KC_YFWD, 2, launch_ypass(st, g, c, t, s0, 1, false, nullptr, nullptr));
        float2 *in[2] = {S[4], S[0]};
        float2 *add0[2] = {S[5], S[6]};
        const double med_units = (ms.het[MED_C0SQ] ? 1 : 0) + (ms.het[MED_NL] ? 1 : 0) +
                                 (ms.het[MED_TA] ? 2 : 0);
        if (s->merged_abs) {
            float2 *s1[1] = {S[1]};
            KW_L(KC_ZABS, 5, launch_zfused(st, g, c, t, ZM_ABSM, in, s1, s->med.ta.scalar * r0nxny,
                                           s->med.tb.scalar, add0));
            KW_L(KC_YINV, 2, launch_ypass(st, g, c, t, s1, 1, true, nullptr, nullptr));
            KW_L(KC_XEOS, 3 + med_units + sens_units,
                 launch_xeos(st, g, c, t, s->med, s->src, s->sen, s->counters, s1,
                             s->buf.rho_total, S[0], true));
        } else {
            float2 *s12[2] = {S[1], S[2]};
            KW_L(KC_ZABS, 6, launch_zfused(st, g, c, t, ZM_ABS, in, s12, r0nxny, 1.0f, add0));
            KW_L(KC_YINV, 4, launch_ypass(st, g, c, t, s12, 2, true, nullptr, nullptr));
            KW_L(KC_XEOS, 4 + med_units + sens_units,
                 launch_xeos(st, g, c, t, s->med, s->src, s->sen, s->counters, s12,
                             s->buf.rho_total, S[0]));
        }
        s->kernels_per_step = nk;
        return hipSuccess;
    }
    KW_L(KC_ZDIV, 6, launch_zfused(st, g, c, t, ZM_DIV, s123, s456));
    KW_L(KC_YINV, 6, launch_ypass(st, g, c, t, s456, 3, true, nullptr, nullptr));
    if (absorbing) {
        float2 *out2[2] = {S[1], S[2]};
        KW_L(KC_XDEN, 12 + (ms.het[MED_RHO0] ? 1 : 0),
             launch_xden(st, g, c, t, s->med, s->src, s->sen, s->counters, s456, s->buf.rho,
                         s->buf.rho_total, out2, false, rec));
        float2 *s12[2] = {S[1], S[2]};
        float2 *s45[2] = {S[4], S[5]};
        KW_L(KC_YFWD, 4, launch_ypass(st, g, c, t, s12, 2, false, nullptr, nullptr));
        const double med_units = (ms.het[MED_C0SQ] ? 1 : 0) + (ms.het[MED_NL] ? 1 : 0) +
                                 (ms.het[MED_TA] ? 2 : 0);
        if (s->merged_abs) {
            // scalar c0^2 tau and c0^2 eta: both terms of Eq. (8) in one spectrum
            KW_L(KC_ZABS, 3, launch_zfused(st, g, c, t, ZM_ABSM, s12, s45, s->med.ta.scalar,
                                           s->med.tb.scalar));
            KW_L(KC_YINV, 2, launch_ypass(st, g, c, t, s45, 1, true, nullptr, nullptr));
            KW_L(KC_XEOS, 3 + med_units + sens_units,
                 launch_xeos(st, g, c, t, s->med, s->src, s->sen, s->counters, s45,
                             s->buf.rho_total, S[0], true));
        } else {
            KW_L(KC_ZABS, 4, launch_zfused(st, g, c, t, ZM_ABS, s12, s45));
            KW_L(KC_YINV, 4, launch_ypass(st, g, c, t, s45, 2, true, nullptr, nullptr));
            KW_L(KC_XEOS, 4 + med_units + sens_units,
                 launch_xeos(st, g, c, t, s->med, s->src, s->sen, s->counters, s45,
                             s->buf.rho_total, S[0]));
        }
    } else {
        float2 *out1[2] = {S[0], nullptr};
        const double med_units = (ms.het[MED_RHO0] ? 1 : 0) + (ms.het[MED_C0SQ] ? 1 : 0) +
                                 (ms.het[MED_NL] ? 1 : 0);
        KW_L(KC_XDEN, 10 + med_units + sens_units,
             launch_xden(st, g, c, t, s->med, s->src, s->sen, s->counters, s456, s->buf.rho,
                         nullptr, out1, false, rec));
    }
#undef KW_L
    s->kernels_per_step = nk;
    return hipSuccess;
}

void drop_graph(kw_sim *s) {
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->graph_exec = nullptr;
    s->graph = nullptr;
}

int build_graph(kw_sim *s) {
    drop_graph(s);
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(KW_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    hipError_t el = hipSuccess;
    for (int i = 0; i < s->graph_steps && el == hipSuccess; ++i) el = enqueue_step(s);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(s->stream, &gr);
    if (el != hipSuccess || e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return fail(KW_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(el != hipSuccess ? el : e));
    }
    s->graph = gr;
    e = hipGraphInstantiate(&s->graph_exec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(s);
        return fail(KW_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return KW_OK;
}

// A block of tb x L threads with `lds` bytes: up to 512 threads and 64 KB, or,
// for the column passes of the fixed engines (`wide`), up to 1024 threads and
// the device's LDS per block.
// wide: 1024-thread instantiations exist (fixed 8- and 16-wide engines);
// big_lds: the block may use all the LDS of a CU (fixed engines but 12, 20)
int check_tb(const char *what, int tb, int L, size_t lds, bool wide = false,
             size_t max_lds = 64 * 1024, bool big_lds = false) {
    const int max_threads = wide ? 1024 : 512;
    const size_t lds_cap = (wide || big_lds) ? max_lds : (size_t)64 * 1024;
    if (tb < 1 || tb * L > max_threads)
        return fail(KW_EUNSUPPORTED, "%s: %d x %d threads exceed a block", what, tb, L);
    if (lds > lds_cap) return fail(KW_EUNSUPPORTED, "%s: %zu bytes of LDS", what, lds);
    return KW_OK;
}

int pick_tiles(kw_sim *s, int tile_y, int tile_z) {
    LaunchCfg &c = s->cfg;
    const GridDev &g = s->g;
    // rows per block in the x kernels: about 256 threads
    c.tb_x = std::max(1, 256 / c.px.L);
    while (c.tb_x > 1 && x_lds_bytes(g.M, g.nx, c.tb_x, true) > 64 * 1024) c.tb_x /= 2;
    // rows per block of the three-group density kernel of the generic
    // engines: as many as fit 512 threads and 64 KB of LDS
    if (!eng_fixed(c.eng_x) || eng_general(c.eng_x) == ENG_F12 || eng_wide(c.eng_x)) {
        const bool line = den_needs_line(s->med, s->src, s->sen);
        auto fits = [&](int tb) {
            return 3 * tb * c.px.L <= 512 && den_lds_bytes(g.M, g.nx, tb, line) <= 64 * 1024;
        };
        int best = 0;
        for (int tb = 1; fits(tb); ++tb) best = tb;
        if (best == 0)
            return fail(KW_EUNSUPPORTED, "density pass does not fit a block (nx = %d)", g.nx);
        c.tb_den = best;
    } else {
        c.tb_den = c.tb_x;
    }
    // columns per block of the y and z passes: 16 (128-byte rows of a tile)
    // where a block can hold them -- for the fixed engines up to 1024 threads
    // and the device's LDS per block (measured at 1024^3: 120 -> 111 ms per
    // step against 8 columns of 512 threads), else 512 threads and 64 KB
    auto col_tile = [&](int n, int L, int req, bool wide, size_t (*bytes)(int, int), bool big = false) {
        if (req > 0) return req;
        const int max_threads = wide ? 1024 : 512;
        const size_t max_bytes = (wide || big) ? s->max_lds : (size_t)64 * 1024;
        int tb = 16;
        while (tb > 1 && (tb * L > max_threads || bytes(n, tb) > max_bytes)) tb /= 2;
        return tb;
    };
    const int gy = eng_general(c.eng_y), gz = eng_general(c.eng_z);
    c.tb_y = col_tile(g.ny, c.py.L, tile_y, gy == ENG_F8 || gy == ENG_F16, col_lds_bytes,
                      c.eng_y == ENG_F32);
    c.tb_z = col_tile(g.nz, c.pz.L, tile_z, gz == ENG_F8 || gz == ENG_F16, zcol_lds_bytes,
                      c.eng_z == ENG_F32);
    int rc;
    if ((rc = check_tb("x pass", c.tb_x, c.px.L, x_lds_bytes(g.M, g.nx, c.tb_x, true))) != KW_OK)
        return rc;
    const bool wide_y = gy == ENG_F8 || gy == ENG_F16;
    const bool wide_z = gz == ENG_F8 || gz == ENG_F16;
    if ((rc = check_tb("y pass", c.tb_y, c.py.L, col_lds_bytes(g.ny, c.tb_y), wide_y,
                       s->max_lds, c.eng_y == ENG_F32)) != KW_OK)
        return rc;
    if ((rc = check_tb("z pass", c.tb_z, c.pz.L, zcol_lds_bytes(g.nz, c.tb_z), wide_z,
                       s->max_lds, c.eng_z == ENG_F32)) != KW_OK)
        return rc;
    // The merged absorption pass holds two spectra per thread and runs at two
    // wavefronts per SIMD with either fixed engine; on 1024-point columns it
    // takes the 32-wide engine's two radix-32 passes in 16-column tiles
    // (measured at 1024^3: 11.5 -> 8.8 ms; the gradient and divergence passes,
    // at four wavefronts on the 16-wide engine, lost with it)
    c.eng_za = c.eng_z;
    c.pza = c.pz;
    c.pzai = c.pzi;
    c.tb_za = c.tb_z;
    if (g.nz == 1024 && gz == ENG_F16) {
        FftPlan f;
        if (fixed_plan_from_radices(1024, 32, {32, 32}, f) && 16 * f.L <= 512 &&
            zcol_lds_bytes(g.nz, 16) <= s->max_lds) {
            c.eng_za = ENG_F32;
            c.pza = c.pzai = f;
            c.tb_za = 16;
        }
    }
    // the column passes address an element of their tile by a 32-bit byte offset
    const uint64_t zlane = ((uint64_t)std::max(c.pz.L, c.pza.L) * g.M * g.ny + std::max(c.tb_z, c.tb_za)) * 8;
    if (zlane >= (1ull << 32))
        return fail(KW_EUNSUPPORTED, "z pass: tile offsets of %llu bytes exceed 32 bits",
                    (unsigned long long)zlane);
    return KW_OK;
}

void release(kw_sim *s) {
    resolve_profile(s);
    drop_graph(s);
    for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
    delete s;
}

}  // namespace

// A prepared set-up: the host state of a simulation (every field of kw_sim
// but its workspace, stream and device pointers) and the bytes to upload.
struct kw_plan {
    kw_sim proto;
    MediumShape ms;
    std::vector<std::pair<size_t, std::vector<char>>> up;   // (workspace offset, bytes)
};

namespace {

// Host part of set-up: validation, FFT plans, float64 tables and per-point
// maps, source and sensor lists.  No HIP call: safe in any thread.
int prepare(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
            const kw_sensor *sensor, kw_plan *P) {
    Counts cnt;
    int rc = validate(grid, medium, source, sensor, cnt);
    if (rc != KW_OK) return rc;
    const Layout L = make_layout(grid, medium, cnt);

    const int nx = grid->nx, ny = grid->ny, nz = grid->nz, M = nx / 2;
    const size_t N = (size_t)nx * ny * nz;
    const double d[3] = {grid->dx, grid->dy, grid->dz};
    const int n3[3] = {nx, ny, nz};

    // FFT plans (host only, may fail before any device work)
    LaunchCfg cfg{};
    if (!axis_plan(M, 0, nullptr, cfg.eng_x, cfg.px, cfg.pxi) ||
        !axis_plan(ny, 1, nullptr, cfg.eng_y, cfg.py, cfg.pyi) ||
        !axis_plan(nz, 2, nullptr, cfg.eng_z, cfg.pz, cfg.pzi))
        return fail(KW_EUNSUPPORTED, "no FFT schedule for %d x %d x %d", nx, ny, nz);

    // medium scalars / statistics in float64
    auto val = [](const float *a, double sc, size_t i) { return a ? (double)a[i] : sc; };
    double cmax = 0.0;
    if (medium->c0) {
        for (size_t i = 0; i < N; ++i) {
            const double c = medium->c0[i];
            if (!(c > 0.0) || !std::isfinite(c)) return fail(KW_EINVAL, "c0[%zu] not positive", i);
            cmax = std::max(cmax, c);
        }
    } else {
        cmax = medium->c0_scalar;
    }
    if (medium->rho0) {
        for (size_t i = 0; i < N; ++i)
            if (!(medium->rho0[i] > 0.0f)) return fail(KW_EINVAL, "rho0[%zu] not positive", i);
    }
    const double c_ref = medium->c_ref > 0.0 ? medium->c_ref : cmax;
    const double dt = grid->dt > 0.0 ? grid->dt
                                     : grid->cfl * std::min({grid->dx, grid->dy, grid->dz}) / cmax;
    const bool nonlinear = medium->flags & KW_NONLINEAR;
    const bool absorbing = medium->flags & KW_ABSORBING;
    const double y = medium->alpha_power;

    kw_sim *s = &P->proto;
    s->grid = *grid;
    s->flags = medium->flags;
    s->L = L;
    s->cnt = cnt;
    s->cfg = cfg;
    s->dt = dt;
    s->c_ref = c_ref;
    s->record_start = sensor ? sensor->record_start : 1;
    GridDev &g = s->g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.M = M;
    g.rows = ny * nz;
    g.inv_n = (float)(1.0 / (double)N);
    g.half_cdt = (float)(0.5 * c_ref * dt);
    g.dt = (float)dt;
    g.y_tau = (float)((y - 2.0) / 2.0);
    g.y_eta = (float)((y - 1.0) / 2.0);
    g.dkz = (float)(2.0 * kPi / (grid->dz * nz));

    auto &up = P->up;   // (workspace offset, bytes)
    auto put = [&](size_t off, const void *p, size_t n) {
        std::vector<char> v((const char *)p, (const char *)p + n);
        up.emplace_back(off, std::move(v));
    };
    auto put_f2 = [&](size_t off, const std::vector<double> &re, const std::vector<double> &im) {
        std::vector<float2> v(re.size());
        for (size_t i = 0; i < re.size(); ++i) v[i] = make_float2((float)re[i], (float)im[i]);
        put(off, v.data(), v.size() * sizeof(float2));
    };
    auto put_f = [&](size_t off, const std::vector<double> &a) {
        std::vector<float> v(a.begin(), a.end());
        put(off, v.data(), v.size() * sizeof(float));
    };

    // twiddles
    {
        std::vector<double> re(M), im(M);
        for (int m = 0; m < M; ++m) {
            re[m] = std::cos(2.0 * kPi * m / M);
            im[m] = -std::sin(2.0 * kPi * m / M);
        }
        put_f2(L.tw_x, re, im);
        for (int k = 0; k < M; ++k) {
            re[k] = std::cos(2.0 * kPi * k / nx);
            im[k] = -std::sin(2.0 * kPi * k / nx);
        }
        put_f2(L.tw_post, re, im);
        for (int a = 1; a < 3; ++a) {
            const int n = n3[a];
            std::vector<double> r2(n), i2(n);
            for (int m = 0; m < n; ++m) {
                r2[m] = std::cos(2.0 * kPi * m / n);
                i2[m] = -std::sin(2.0 * kPi * m / n);
            }
            put_f2(a == 1 ? L.tw_y : L.tw_z, r2, i2);
        }
    }
    // wavenumbers and shift operators i k exp(+-i k d / 2) (Eqs. (4a), (4c), (5))
    for (int a = 0; a < 3; ++a) {
        const int n = n3[a];
        const int len = (a == 0) ? M + 1 : n;
        std::vector<double> k(len), pr(len), pi(len), mr(len), mi(len);
        for (int j = 0; j < len; ++j) {
            k[j] = wavenumber(j, n, d[a]);
            const double h = k[j] * d[a] / 2.0;
            pr[j] = -k[j] * std::sin(h);
            pi[j] = k[j] * std::cos(h);
            mr[j] = k[j] * std::sin(h);
            mi[j] = k[j] * std::cos(h);
            if (n % 2 == 0 && j == n / 2) pi[j] = mi[j] = 0.0;   // Nyquist: exactly real
        }
        const size_t ko[3] = {L.kx, L.ky, L.kz};
        const size_t po[3] = {L.dpx, L.dpy, L.dpz};
        const size_t mo[3] = {L.dmx, L.dmy, L.dmz};
        put_f(ko[a], k);
        put_f2(po[a], pr, pi);
        put_f2(mo[a], mr, mi);
    }
    // PML
    for (int a = 0; a < 3; ++a) {
        const int n = n3[a];
        std::vector<double> r(n), sg(n);
        for (int i = 0; i < n; ++i) {
            r[i] = pml_factor(i, false, n, grid->pml_size[a], grid->pml_alpha[a], c_ref, d[a], dt);
            sg[i] = pml_factor(i, true, n, grid->pml_size[a], grid->pml_alpha[a], c_ref, d[a], dt);
        }
        put_f(L.pml[2 * a], r);
        put_f(L.pml[2 * a + 1], sg);
    }

    // medium coefficients
    const double np_per_db = 100.0 / (20.0 * std::log10(std::exp(1.0))) /
                             std::pow(2.0 * kPi * 1.0e6, y);
    const double tan_y = std::tan(kPi * y / 2.0);
    const MediumShape ms = medium_shape(medium);
    P->ms = ms;
    auto c0_at = [&](size_t i) { return val(medium->c0, medium->c0_scalar, i); };
    auto rho_at = [&](size_t i) { return val(medium->rho0, medium->rho0_scalar, i); };
    auto a_at = [&](size_t i) { return val(medium->alpha0, medium->alpha0_scalar, i) * np_per_db; };
    auto b_at = [&](size_t i) { return val(medium->bona, medium->bona_scalar, i); };
    auto tau_at = [&](size_t i) { return -2.0 * a_at(i) * std::pow(c0_at(i), y - 1.0); };
    auto eta_at = [&](size_t i) { return 2.0 * a_at(i) * std::pow(c0_at(i), y) * tan_y; };
    auto stag_rho = [&](int axis, size_t i) {
        const size_t stride = axis == 0 ? 1 : axis == 1 ? (size_t)nx : (size_t)nx * ny;
        const int coord = axis == 0 ? (int)(i % nx) : axis == 1 ? (int)((i / nx) % ny)
                                                                : (int)(i / ((size_t)nx * ny));
        if (coord == n3[axis] - 1) return rho_at(i);
        return 0.5 * (rho_at(i) + rho_at(i + stride));
    };
    Medium &md = s->med;
    md.nonlinear = nonlinear;
    md.absorbing = absorbing;
    s->merged_abs = absorbing && !ms.het[MED_TA];
    s->rho0_sum_in_z = absorbing && !ms.het[MED_RHO0];
    {
        auto fill_map = [&](int which, auto fn, Coef &dst) {
            if (ms.het[which]) {
                std::vector<float> v(N);
                for (size_t i = 0; i < N; ++i) v[i] = (float)fn(i);
                put(L.med[which], v.data(), N * sizeof(float));
                dst.map = nullptr;              // set when the workspace is bound
                dst.scalar = 0.0f;
            } else {
                dst.map = nullptr;
                dst.scalar = (float)fn(0);
            }
        };
        for (int a = 0; a < 3; ++a)
            fill_map(MED_DTRX + a, [&](size_t i) { return dt / stag_rho(a, i); }, md.dtr[a]);
        fill_map(MED_RHO0, [&](size_t i) { return rho_at(i); }, md.rho0);
        fill_map(MED_C0SQ, [&](size_t i) { return c0_at(i) * c0_at(i); }, md.c0sq);
        fill_map(MED_NL, [&](size_t i) {
            return nonlinear ? c0_at(i) * c0_at(i) * b_at(i) / (2.0 * rho_at(i)) : 0.0; }, md.nl);
        fill_map(MED_TA, [&](size_t i) {
            return absorbing ? c0_at(i) * c0_at(i) * tau_at(i) : 0.0; }, md.ta);
        fill_map(MED_TB, [&](size_t i) {
            return absorbing ? -c0_at(i) * c0_at(i) * eta_at(i) : 0.0; }, md.tb);
    }

    // source
    SourceDev &sd = s->src;
    if (cnt.n_src > 0) {
        const long ns = cnt.n_src;
        const int rows = ny * nz;
        std::vector<int> rp(rows + 1, 0), xp(ns), el(ns);
        std::vector<float> cf(ns);
        for (long i = 0; i < ns; ++i) {
            const long idx = source->index[i];
            rp[idx / nx + 1]++;
            xp[i] = (int)(idx % nx);
            el[i] = source->element ? source->element[i] : 0;
            // mass: dt M_xi per unit drive; force: dt; pressure: the drive itself
            cf[i] = source->kind == KW_SOURCE_MASS
                        ? (float)(2.0 * dt / (3.0 * c0_at((size_t)idx) * grid->dx))
                        : source->kind == KW_SOURCE_FORCE ? (float)dt : 1.0f;
        }
        for (int r = 0; r < rows; ++r) rp[r + 1] += rp[r];
        std::vector<double> ac(cnt.n_elem), as(cnt.n_elem);
        for (int e = 0; e < cnt.n_elem; ++e) {
            ac[e] = (double)source->amp[e] * std::cos((double)source->phase[e]);
            as[e] = (double)source->amp[e] * std::sin((double)source->phase[e]);
        }
        put(L.src_row, rp.data(), rp.size() * sizeof(int));
        put(L.src_x, xp.data(), ns * sizeof(int));
        put(L.src_e, el.data(), ns * sizeof(int));
        put(L.src_c, cf.data(), ns * sizeof(float));
        put(L.src_ac, ac.data(), ac.size() * sizeof(double));
        put(L.src_as, as.data(), as.size() * sizeof(double));
        sd.n_elements = cnt.n_elem;
        sd.omega_dt = 2.0 * kPi * source->freq * dt;
        sd.kind = source->kind;
        sd.axis = source->kind == KW_SOURCE_FORCE ? source->axis : 0;
        sd.t_offset = source->kind == KW_SOURCE_MASS ? 0.5 : source->kind == KW_SOURCE_FORCE ? 0.0 : 1.0;
        s->src_flat.resize(ns);
        for (long i = 0; i < ns; ++i) s->src_flat[i] = (int)source->index[i];
        s->src_elem = el;
        s->src_coef = cf;
        s->src_amp.assign(source->amp, source->amp + cnt.n_elem);
        s->src_phase.assign(source->phase, source->phase + cnt.n_elem);
        if (cnt.n_samples > 0) {
            put(L.src_sig, source->signal, (size_t)cnt.n_elem * cnt.n_samples * sizeof(float));
            sd.n_samples = cnt.n_samples;
        }
    }

    // sensor
    SensorDev &se = s->sen;
    se.all_points = cnt.sen_all ? 1 : 0;
    se.record_start = s->record_start;
    se.capacity = cnt.capacity;
    if (!cnt.sen_all && cnt.n_sen > 0) {
        const long nsn = cnt.n_sen;
        const int rows = ny * nz;
        std::vector<int> rp(rows + 1, 0), xp(nsn), id(nsn), ix(nsn);
        for (long i = 0; i < nsn; ++i) {
            const long idx = sensor->index[i];
            rp[idx / nx + 1]++;
            xp[i] = (int)(idx % nx);
            id[i] = (int)i;
            ix[i] = (int)idx;
        }
        for (int r = 0; r < rows; ++r) rp[r + 1] += rp[r];
        put(L.sen_row, rp.data(), rp.size() * sizeof(int));
        put(L.sen_x, xp.data(), nsn * sizeof(int));
        put(L.sen_id, id.data(), nsn * sizeof(int));
        put(L.sen_idx, ix.data(), nsn * sizeof(int));
        se.n_points = (int)nsn;
    } else {
        se.n_points = cnt.sen_all ? (int)N : 0;
    }
    if (L.harm) {
        se.n_harm = cnt.n_harm;
        se.harm_wdt = 2.0 * kPi * cnt.harm_freq * dt;
    }

    return KW_OK;
}

// Point the simulation's device arrays into its workspace (s->ws): the
// per-point maps the medium needs, source and sensor lists, accumulators,
// 1D tables, counters and the state and spectral arrays.
void bind(kw_sim *s, const MediumShape &ms) {
    const Layout &L = s->L;
    const Counts &cnt = s->cnt;
    Medium &md = s->med;
    Coef *maps[8] = {&md.dtr[0], &md.dtr[1], &md.dtr[2], &md.rho0,
                     &md.c0sq,   &md.nl,     &md.ta,     &md.tb};
    for (int i = 0; i < 8; ++i) maps[i]->map = ms.het[i] ? s->at<float>(L.med[i]) : nullptr;
    SourceDev &sd = s->src;
    sd.drive = s->at<float>(L.drive);
    if (cnt.n_src > 0) {
        sd.row_ptr = s->at<int>(L.src_row);
        sd.xpos = s->at<int>(L.src_x);
        sd.elem = s->at<int>(L.src_e);
        sd.coef = s->at<float>(L.src_c);
        sd.amp_cos = s->at<double>(L.src_ac);
        sd.amp_sin = s->at<double>(L.src_as);
        if (cnt.n_samples > 0) sd.signal = s->at<float>(L.src_sig);
    }
    SensorDev &se = s->sen;
    if (!cnt.sen_all && cnt.n_sen > 0) {
        se.row_ptr = s->at<int>(L.sen_row);
        se.xpos = s->at<int>(L.sen_x);
        se.sid = s->at<int>(L.sen_id);
    }
    if (L.p_max) se.p_max = s->at<float>(L.p_max);
    if (L.p_sum2) se.p_sum2 = s->at<float>(L.p_sum2);
    if (L.series) se.series = s->at<float>(L.series);
    if (L.p_min) se.p_min = s->at<float>(L.p_min);
    if (L.harm) {
        se.harm = s->at<float>(L.harm);
        se.hw = s->at<float>(L.hw);
    }
    if (L.useries) se.u_series = s->at<float>(L.useries);

    // tables
    Tables &t = s->tab;
    t.tw_x = s->at<float2>(L.tw_x);
    t.tw_post = s->at<float2>(L.tw_post);
    t.tw_y = s->at<float2>(L.tw_y);
    t.tw_z = s->at<float2>(L.tw_z);
    t.kx = s->at<float>(L.kx);
    t.ky = s->at<float>(L.ky);
    t.kz = s->at<float>(L.kz);
    t.dpx = s->at<float2>(L.dpx);
    t.dmx = s->at<float2>(L.dmx);
    t.dpy = s->at<float2>(L.dpy);
    t.dmy = s->at<float2>(L.dmy);
    t.dpz = s->at<float2>(L.dpz);
    t.dmz = s->at<float2>(L.dmz);
    t.pml_x = s->at<float>(L.pml[0]);
    t.pml_sx = s->at<float>(L.pml[1]);
    t.pml_y = s->at<float>(L.pml[2]);
    t.pml_sy = s->at<float>(L.pml[3]);
    t.pml_z = s->at<float>(L.pml[4]);
    t.pml_sz = s->at<float>(L.pml[5]);
    s->counters.step = s->at<int>(L.counters);
    s->counters.nonfinite = s->at<int>(L.counters) + 1;
    for (int i = 0; i < 3; ++i) {
        s->buf.u[i] = s->at<float>(L.u[i]);
        s->buf.rho[i] = s->at<float>(L.rho[i]);
    }
    s->buf.rho_total = L.rho_total ? s->at<float>(L.rho_total) : nullptr;
    for (int i = 0; i < 7; ++i) s->buf.S[i] = s->at<float2>(L.S[i]);

}

// Device part of set-up: bind a prepared plan to a workspace and a stream,
// choose the launch shapes, upload the tables and maps, zero the state.
// With `static_spectra` the six spectral scratch arrays S1..S6 (the last
// regions of the layout) come from the library's static scratch array and the
// workspace ends where S1 would start.
int create_prepared(const kw_plan *P, void *dev_workspace, size_t ws_bytes, void *stream,
                    kw_sim **out, bool static_spectra = false) {
    if (!out) return fail(KW_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!P) return fail(KW_EINVAL, "plan must not be NULL");
    const Layout &L = P->proto.L;
    const size_t need = static_spectra ? L.S[1] : L.total;
    if (!dev_workspace) return fail(KW_EINVAL, "workspace must not be NULL");
    if ((reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) != 0)
        return fail(KW_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (ws_bytes < need)
        return fail(KW_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    char *spectra = nullptr;
    if (static_spectra) {
        void *p = nullptr;
        size_t cap = 0;
        const hipError_t e = static_scratch(&p, &cap);
        if (e != hipSuccess)
            return fail(KW_EDEVICE, "static scratch address: %s", hipGetErrorString(e));
        if (L.total - L.S[1] > cap)
            return fail(KW_EUNSUPPORTED,
                        "the six spectral scratch arrays need %zu bytes, the static scratch "
                        "array holds %zu", L.total - L.S[1], cap);
        spectra = reinterpret_cast<char *>(p);
    }
    kw_sim *s = new (std::nothrow) kw_sim(P->proto);
    if (!s) return fail(KW_EINVAL, "out of host memory");
    s->stream = reinterpret_cast<hipStream_t>(stream);
    s->ws = reinterpret_cast<char *>(dev_workspace);
    s->ws_used = need;
    if (s->stream == nullptr) s->graph_steps = 0;   // the legacy stream cannot be captured
    bind(s, P->ms);
    if (spectra)
        for (int i = 1; i < 7; ++i)
            s->buf.S[i] = reinterpret_cast<float2 *>(spectra + (L.S[i] - L.S[1]));
    const Counts &cnt = s->cnt;
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    SensorDev &se = s->sen;
    SourceDev &sd = s->src;
    int rc;

    // launch shapes (they depend on the source and sensor set-up above)
    {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            s->max_lds = (size_t)v;
        (void)hipGetLastError();
    }
    if ((rc = pick_tiles(s, 0, 0)) != KW_OK) {
        delete s;
        return rc;
    }

    // device work: uploads, then zero the state
    auto bail = [&](int code) {
        release(s);
        return code;
    };
    int dev_count = 0;
    if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1)
        return bail(fail(KW_EDEVICE, "no HIP device"));
    for (auto &u : P->up) {
        hipError_t e = hipMemcpyAsync(s->ws + u.first, u.second.data(), u.second.size(),
                                      hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return bail(fail(KW_EDEVICE, "upload: %s", hipGetErrorString(e)));
    }
    hipError_t e = hipSuccess;
    auto z = [&](float *p, size_t n, float v) {
        if (p && e == hipSuccess) e = launch_fill(s->stream, p, n, v);
    };
    for (int i = 0; i < 3; ++i) {
        z(s->buf.u[i], N, 0.0f);
        z(s->buf.rho[i], N, 0.0f);
    }
    z(s->buf.rho_total, N, 0.0f);
    z(reinterpret_cast<float *>(s->buf.S[0]), N, 0.0f);
    const size_t nrec = cnt.sen_all ? N : (size_t)cnt.n_sen;
    z(se.p_max, nrec, -INFINITY);
    z(se.p_sum2, nrec, 0.0f);
    z(se.series, (size_t)cnt.capacity * cnt.n_sen, 0.0f);
    z(se.p_min, nrec, INFINITY);
    z(se.harm, (size_t)2 * cnt.n_harm * nrec, 0.0f);
    z(se.hw, (size_t)2 * cnt.n_harm, 0.0f);
    z(se.u_series, (size_t)cnt.capacity * 3 * cnt.n_sen, 0.0f);
    z(sd.drive, std::max(1, cnt.n_elem), 0.0f);
    if (e == hipSuccess) e = launch_fill_int(s->stream, s->counters.step, 1, 0);
    if (e == hipSuccess) e = launch_fill_int(s->stream, s->counters.nonfinite, 1, INT_MAX);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(fail(KW_EDEVICE, "initialisation: %s", hipGetErrorString(e)));
    *out = s;
    return KW_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *kw_last_error(void) { return g_err.c_str(); }

size_t kw_workspace_size(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
                         const kw_sensor *sensor) {
    Counts c;
    if (validate(grid, medium, source, sensor, c) != KW_OK) return 0;
    return make_layout(grid, medium, c).total;
}

int kw_prepare(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
               const kw_sensor *sensor, kw_plan **out) {
    if (!out) return fail(KW_EINVAL, "out must not be NULL");
    *out = nullptr;
    kw_plan *P = new (std::nothrow) kw_plan();   // value-initialised (zeroed structs)
    if (!P) return fail(KW_EINVAL, "out of host memory");
    const int rc = prepare(grid, medium, source, sensor, P);
    if (rc != KW_OK) {
        delete P;
        return rc;
    }
    *out = P;
    return KW_OK;
}

size_t kw_plan_workspace_size(const kw_plan *plan) { return plan ? plan->proto.L.total : 0; }

int kw_create_prepared(const kw_plan *plan, void *dev_workspace, size_t ws_bytes, void *stream,
                       kw_sim **out) {
    return create_prepared(plan, dev_workspace, ws_bytes, stream, out);
}

int kw_create_static(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
                     const kw_sensor *sensor, void *dev_workspace, size_t ws_bytes, void *stream,
                     kw_sim **out) {
    if (!out) return fail(KW_EINVAL, "out must not be NULL");
    *out = nullptr;
    kw_plan P{};
    const int rc = prepare(grid, medium, source, sensor, &P);
    if (rc != KW_OK) return rc;
    return create_prepared(&P, dev_workspace, ws_bytes, stream, out, true);
}

int kw_plan_destroy(kw_plan *plan) {
    delete plan;
    return KW_OK;
}

int kw_create(const kw_grid *grid, const kw_medium *medium, const kw_source *source,
              const kw_sensor *sensor, void *dev_workspace, size_t ws_bytes, void *stream,
              kw_sim **out) {
    if (!out) return fail(KW_EINVAL, "out must not be NULL");
    *out = nullptr;
    kw_plan P{};   // value-initialised: the plain structs of the prototype start zeroed
    const int rc = prepare(grid, medium, source, sensor, &P);
    if (rc != KW_OK) return rc;
    return create_prepared(&P, dev_workspace, ws_bytes, stream, out);
}

int kw_step(kw_sim *s, int32_t n) {
    if (!s) return fail(KW_EINVAL, "sim is NULL");
    if (n < 0) return fail(KW_EINVAL, "n must be >= 0");
    long done = 0;
    const bool use_graph = s->graph_steps > 0 && !s->profiling;
    if (use_graph && n >= s->graph_steps) {
        if (!s->graph_exec) {
            int rc = build_graph(s);
            if (rc != KW_OK) return rc;
        }
        while (n - done >= s->graph_steps) {
            hipError_t e = hipGraphLaunch(s->graph_exec, s->stream);
            if (e != hipSuccess) return fail(KW_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
            done += s->graph_steps;
        }
    }
    for (; done < n; ++done) {
        hipError_t e = enqueue_step(s);
        if (e != hipSuccess) return fail(KW_EDEVICE, "kernel launch: %s", hipGetErrorString(e));
    }
    s->steps += n;
    s->stepped = s->stepped || n > 0;
    return KW_OK;
}

int64_t kw_gather_bytes(kw_sim *s, uint32_t what) {
    if (!s) return -1;
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    const size_t nrec = s->cnt.sen_all ? N : (size_t)s->cnt.n_sen;
    switch (what) {
    case KW_REC_P_MAX:
    case KW_REC_P_MIN:
    case KW_REC_P_RMS:
    case KW_REC_INTENSITY:
        return (int64_t)(nrec * sizeof(float));
    case KW_REC_HARMONICS:
        return (int64_t)((size_t)2 * s->cnt.n_harm * nrec * sizeof(float));
    case KW_REC_U_SERIES: {
        const long rec = std::max(0L, s->steps - s->record_start + 1);
        return (int64_t)(std::min<long>(rec, s->cnt.capacity) * 3 * s->cnt.n_sen * sizeof(float));
    }
    case KW_REC_P_SERIES: {
        const long rec = std::max(0L, s->steps - s->record_start + 1);
        return (int64_t)(std::min<long>(rec, s->cnt.capacity) * s->cnt.n_sen * sizeof(float));
    }
    case KW_REC_P_FINAL:
        return (int64_t)(N * sizeof(float));
    case KW_REC_U_FINAL:
        return (int64_t)(3 * N * sizeof(float));
    default:
        return -1;
    }
}

static int copy_out(kw_sim *s, void *dst, const void *src, size_t n, int dst_is_device) {
    KW_HIP(hipMemcpyAsync(dst, src, n, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          s->stream));
    return KW_OK;
}

int kw_gather(kw_sim *s, uint32_t what, void *dst, size_t dst_bytes, int dst_is_device) {
    if (!s || !dst) return fail(KW_EINVAL, "NULL argument");
    const int64_t need = kw_gather_bytes(s, what);
    if (need < 0) return fail(KW_EINVAL, "unknown gather target %u", what);
    if (!(what & (s->cnt.record | KW_REC_P_FINAL | KW_REC_U_FINAL)))
        return fail(KW_EINVAL, "quantity %u was not recorded", what);
    if ((size_t)need > dst_bytes)
        return fail(KW_EINVAL, "dst has %zu bytes, %lld needed", dst_bytes, (long long)need);
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    const size_t nrec = s->cnt.sen_all ? N : (size_t)s->cnt.n_sen;
    float *tmp = reinterpret_cast<float *>(s->buf.S[1]);   // free between steps
    const long nrec_steps = std::max(0L, s->steps - s->record_start + 1);
    int rc = KW_OK;
    switch (what) {
    case KW_REC_P_MAX:
        rc = copy_out(s, dst, s->sen.p_max, need, dst_is_device);
        break;
    case KW_REC_P_MIN:
        rc = copy_out(s, dst, s->sen.p_min, need, dst_is_device);
        break;
    case KW_REC_U_SERIES:
        if (need > 0) rc = copy_out(s, dst, s->sen.u_series, need, dst_is_device);
        break;
    case KW_REC_HARMONICS: {
        // A_h = (2 / N) times the accumulated sums
        const float scale = nrec_steps > 0 ? (float)(2.0 / nrec_steps) : 0.0f;
        const size_t n = (size_t)need / sizeof(float);
        if (dst_is_device) {
            hipError_t e = launch_scale(s->stream, s->sen.harm, reinterpret_cast<float *>(dst), n,
                                        scale);
            if (e != hipSuccess) return fail(KW_EDEVICE, "scale: %s", hipGetErrorString(e));
        } else {
            rc = copy_out(s, dst, s->sen.harm, need, 0);
            if (rc == KW_OK) {
                KW_HIP(hipStreamSynchronize(s->stream));
                float *h = reinterpret_cast<float *>(dst);
                for (size_t i = 0; i < n; ++i) h[i] *= scale;
            }
        }
        break;
    }
    case KW_REC_P_RMS:
    case KW_REC_INTENSITY: {
        float *target = dst_is_device ? reinterpret_cast<float *>(dst) : tmp;
        const float inv = nrec_steps > 0 ? (float)(1.0 / nrec_steps) : 0.0f;
        hipError_t e = launch_finalize(s->stream, s->sen.p_sum2, target, nrec, inv,
                                       what == KW_REC_P_RMS ? 0 : 1, s->med.rho0, s->med.c0sq,
                                       s->cnt.sen_all ? nullptr : s->at<int>(s->L.sen_idx));
        if (e != hipSuccess) return fail(KW_EDEVICE, "finalize: %s", hipGetErrorString(e));
        if (!dst_is_device) rc = copy_out(s, dst, tmp, need, 0);
        break;
    }
    case KW_REC_P_SERIES:
        if (need > 0) rc = copy_out(s, dst, s->sen.series, need, dst_is_device);
        break;
    case KW_REC_P_FINAL: {
        float *target = dst_is_device ? reinterpret_cast<float *>(dst) : tmp;
        hipError_t e = launch_xinv(s->stream, s->g, s->cfg, s->tab, s->buf.S[0], target,
                                   1.0f / (float)s->grid.nx);
        if (e != hipSuccess) return fail(KW_EDEVICE, "xinv: %s", hipGetErrorString(e));
        if (!dst_is_device) rc = copy_out(s, dst, tmp, need, 0);
        break;
    }
    case KW_REC_U_FINAL:
        for (int i = 0; i < 3 && rc == KW_OK; ++i)
            rc = copy_out(s, reinterpret_cast<char *>(dst) + i * N * sizeof(float), s->buf.u[i],
                          N * sizeof(float), dst_is_device);
        break;
    }
    if (rc != KW_OK) return rc;
    int flag = INT_MAX;
    KW_HIP(hipMemcpyAsync(&flag, s->counters.nonfinite, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    KW_HIP(hipStreamSynchronize(s->stream));
    if (flag != INT_MAX) return fail(KW_ENONFINITE, "non-finite pressure at step %d", flag);
    return KW_OK;
}

int kw_set_field(kw_sim *s, int field, const void *src, int src_is_device) {
    if (!s || !src) return fail(KW_EINVAL, "NULL argument");
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    const hipMemcpyKind kind = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    float *dst = nullptr;
    switch (field) {
    case KW_FIELD_P: {
        float *tmp = reinterpret_cast<float *>(s->buf.S[1]);
        KW_HIP(hipMemcpyAsync(tmp, src, N * sizeof(float), kind, s->stream));
        KW_HIP(launch_xfwd(s->stream, s->g, s->cfg, s->tab, tmp, s->buf.S[0]));
        KW_HIP(hipStreamSynchronize(s->stream));
        return KW_OK;
    }
    case KW_FIELD_UX: case KW_FIELD_UY: case KW_FIELD_UZ:
        dst = s->buf.u[field - KW_FIELD_UX];
        break;
    case KW_FIELD_RHOX: case KW_FIELD_RHOY: case KW_FIELD_RHOZ:
        dst = s->buf.rho[field - KW_FIELD_RHOX];
        break;
    default:
        return fail(KW_EINVAL, "unknown field %d", field);
    }
    KW_HIP(hipMemcpyAsync(dst, src, N * sizeof(float), kind, s->stream));
    KW_HIP(hipStreamSynchronize(s->stream));
    return KW_OK;
}

int kw_gather_field(kw_sim *s, int field, void *dst, int dst_is_device) {
    if (!s || !dst) return fail(KW_EINVAL, "NULL argument");
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    const float *src = nullptr;
    switch (field) {
    case KW_FIELD_P:
        return kw_gather(s, KW_REC_P_FINAL, dst, N * sizeof(float), dst_is_device);
    case KW_FIELD_UX: case KW_FIELD_UY: case KW_FIELD_UZ:
        src = s->buf.u[field - KW_FIELD_UX];
        break;
    case KW_FIELD_RHOX: case KW_FIELD_RHOY: case KW_FIELD_RHOZ:
        src = s->buf.rho[field - KW_FIELD_RHOX];
        break;
    default:
        return fail(KW_EINVAL, "unknown field %d", field);
    }
    int rc = copy_out(s, dst, src, N * sizeof(float), dst_is_device);
    if (rc != KW_OK) return rc;
    KW_HIP(hipStreamSynchronize(s->stream));
    return KW_OK;
}

int kw_profile(kw_sim *s, int on) {
    if (!s) return fail(KW_EINVAL, "sim is NULL");
    if (!on) resolve_profile(s);
    s->profiling = on != 0;
    return KW_OK;
}

int kw_stats(kw_sim *s, kw_stats_t *out) {
    if (!s || !out) return fail(KW_EINVAL, "NULL argument");
    resolve_profile(s);
    std::memset(out, 0, sizeof *out);
    out->steps = s->steps;
    int flag = INT_MAX;
    KW_HIP(hipMemcpyAsync(&flag, s->counters.nonfinite, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    KW_HIP(hipStreamSynchronize(s->stream));
    out->nonfinite_step = flag == INT_MAX ? -1 : flag;
    out->dt = s->dt;
    out->c_ref = s->c_ref;
    out->workspace_bytes = (int64_t)s->ws_used;
    out->fft_forward_per_step = s->med.absorbing ? (s->rho0_sum_in_z ? 5 : 6) : 4;
    out->fft_inverse_per_step = s->med.absorbing ? (s->merged_abs ? 7 : 8) : 6;
    out->kernels_per_step = s->kernels_per_step;
    out->n_classes = KC_COUNT;
    for (int i = 0; i < KC_COUNT; ++i) {
        std::snprintf(out->class_name[i], sizeof out->class_name[i], "%s", kClassNames[i]);
        out->class_ms[i] = s->class_ms[i];
        out->class_launches[i] = s->class_n[i];
        out->class_bytes[i] = s->class_n[i] > 0 ? s->class_bytes[i] / (double)s->class_n[i] : 0.0;
    }
    return KW_OK;
}

int kw_set_graph(kw_sim *s, int32_t steps_per_graph) {
    if (!s) return fail(KW_EINVAL, "sim is NULL");
    if (steps_per_graph < 0) return fail(KW_EINVAL, "steps_per_graph must be >= 0");
    if (s->stream == nullptr && steps_per_graph > 0)
        return fail(KW_ESTATE, "graphs need a non-default stream");
    drop_graph(s);
    s->graph_steps = steps_per_graph;
    return KW_OK;
}

int kw_set_plan(kw_sim *s, int axis, const int32_t *radices, int32_t n_radices, int32_t tile) {
    if (!s) return fail(KW_EINVAL, "sim is NULL");
    if (axis < 0 || axis > 2) return fail(KW_EINVAL, "axis must be 0, 1 or 2");
    if (s->stepped) return fail(KW_ESTATE, "plans are fixed after the first step");
    LaunchCfg save = s->cfg;
    const int n = axis == 0 ? s->g.M : axis == 1 ? s->g.ny : s->g.nz;
    if (radices && n_radices > 0) {
        std::vector<int> rad(radices, radices + n_radices);
        FftPlan f, r;
        int eng;
        if (!axis_plan(n, axis, &rad, eng, f, r))
            return fail(KW_EINVAL, "radices do not form a schedule for length %d", n);
        (axis == 0 ? s->cfg.px : axis == 1 ? s->cfg.py : s->cfg.pz) = f;
        (axis == 0 ? s->cfg.pxi : axis == 1 ? s->cfg.pyi : s->cfg.pzi) = r;
        (axis == 0 ? s->cfg.eng_x : axis == 1 ? s->cfg.eng_y : s->cfg.eng_z) = eng;
    }
    int rc = pick_tiles(s, axis == 1 ? tile : s->cfg.tb_y, axis == 2 ? tile : s->cfg.tb_z);
    if (rc == KW_OK && axis == 0 && tile > 0) {
        s->cfg.tb_x = tile;
        rc = check_tb("x pass", tile, s->cfg.px.L, x_lds_bytes(s->g.M, s->g.nx, tile, true));
    }
    if (rc != KW_OK) {
        s->cfg = save;
        return rc;
    }
    drop_graph(s);
    return KW_OK;
}

// --- state snapshots ----------------------------------------------------------

namespace {

struct StateHeader {
    char magic[8];           // "KWSTATE1"
    int32_t nx, ny, nz;
    uint32_t flags, record;
    int32_t capacity, record_start;
    int64_t n_sensor, steps, payload;
    double dt, c_ref;
};

// device regions of the evolving state, in snapshot order
std::vector<std::pair<void *, size_t>> state_regions(kw_sim *s) {
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    const size_t nrec = s->cnt.sen_all ? N : (size_t)s->cnt.n_sen;
    std::vector<std::pair<void *, size_t>> r;
    r.emplace_back(s->counters.step, 2 * sizeof(int));
    for (int i = 0; i < 3; ++i) r.emplace_back(s->buf.u[i], N * sizeof(float));
    for (int i = 0; i < 3; ++i) r.emplace_back(s->buf.rho[i], N * sizeof(float));
    r.emplace_back(s->buf.S[0], N * sizeof(float));      // x/y/z-packed spectrum of p
    if (s->sen.p_max) r.emplace_back(s->sen.p_max, nrec * sizeof(float));
    if (s->sen.p_sum2) r.emplace_back(s->sen.p_sum2, nrec * sizeof(float));
    if (s->sen.series)
        r.emplace_back(s->sen.series, (size_t)s->cnt.capacity * s->cnt.n_sen * sizeof(float));
    if (s->sen.p_min) r.emplace_back(s->sen.p_min, nrec * sizeof(float));
    if (s->sen.harm)
        r.emplace_back(s->sen.harm, (size_t)2 * s->cnt.n_harm * nrec * sizeof(float));
    if (s->sen.u_series)
        r.emplace_back(s->sen.u_series, (size_t)s->cnt.capacity * 3 * s->cnt.n_sen * sizeof(float));
    return r;
}

StateHeader make_header(kw_sim *s) {
    StateHeader h{};
    std::memcpy(h.magic, "KWSTATE1", 8);
    h.nx = s->grid.nx;
    h.ny = s->grid.ny;
    h.nz = s->grid.nz;
    h.flags = s->flags;
    h.record = s->cnt.record;
    h.capacity = s->cnt.capacity;
    h.record_start = s->record_start;
    h.n_sensor = s->cnt.sen_all ? -1 : s->cnt.n_sen;
    h.steps = s->steps;
    h.dt = s->dt;
    h.c_ref = s->c_ref;
    for (auto &r : state_regions(s)) h.payload += (int64_t)r.second;
    return h;
}

}  // namespace

int64_t kw_state_bytes(kw_sim *s) {
    if (!s) return -1;
    return (int64_t)sizeof(StateHeader) + make_header(s).payload;
}

int kw_save(kw_sim *s, void *dst, size_t dst_bytes, int dst_is_device) {
    if (!s || !dst) return fail(KW_EINVAL, "NULL argument");
    const StateHeader h = make_header(s);
    const size_t need = sizeof h + (size_t)h.payload;
    if (dst_bytes < need) return fail(KW_EINVAL, "dst has %zu bytes, %zu needed", dst_bytes, need);
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    char *d = reinterpret_cast<char *>(dst);
    KW_HIP(hipStreamSynchronize(s->stream));
    if (dst_is_device) KW_HIP(hipMemcpy(d, &h, sizeof h, hipMemcpyHostToDevice));
    else std::memcpy(d, &h, sizeof h);
    size_t off = sizeof h;
    for (auto &r : state_regions(s)) {
        KW_HIP(hipMemcpyAsync(d + off, r.first, r.second, kind, s->stream));
        off += r.second;
    }
    KW_HIP(hipStreamSynchronize(s->stream));
    return KW_OK;
}

int kw_load(kw_sim *s, const void *src, size_t src_bytes, int src_is_device) {
    if (!s || !src) return fail(KW_EINVAL, "NULL argument");
    StateHeader h{};
    if (src_bytes < sizeof h) return fail(KW_EINVAL, "snapshot too small");
    const char *p = reinterpret_cast<const char *>(src);
    KW_HIP(hipStreamSynchronize(s->stream));
    if (src_is_device) KW_HIP(hipMemcpy(&h, p, sizeof h, hipMemcpyDeviceToHost));
    else std::memcpy(&h, p, sizeof h);
    const StateHeader me = make_header(s);
    if (std::memcmp(h.magic, me.magic, 8) != 0) return fail(KW_EINVAL, "not a kw state snapshot");
    if (h.nx != me.nx || h.ny != me.ny || h.nz != me.nz || h.flags != me.flags ||
        h.record != me.record || h.capacity != me.capacity || h.record_start != me.record_start ||
        h.n_sensor != me.n_sensor || h.payload != me.payload || h.dt != me.dt || h.c_ref != me.c_ref)
        return fail(KW_EINVAL, "snapshot was taken from a simulation with another set-up");
    if (src_bytes < sizeof h + (size_t)h.payload)
        return fail(KW_EINVAL, "snapshot truncated: %zu of %zu bytes", src_bytes,
                    sizeof h + (size_t)h.payload);
    const hipMemcpyKind kind = src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    size_t off = sizeof h;
    for (auto &r : state_regions(s)) {
        KW_HIP(hipMemcpyAsync(r.first, p + off, r.second, kind, s->stream));
        off += r.second;
    }
    KW_HIP(hipStreamSynchronize(s->stream));
    s->steps = h.steps;
    return KW_OK;
}

// --- reverse mode ---------------------------------------------------------------

struct kw_adj {
    kw_sim *sim = nullptr;
    AdjDev a{};
    int n_steps = 0;
};

namespace {

struct AdjLayout {
    size_t fld[12];          // pb, ub x3, rb x3, d x3, w, rbt
    size_t dJds, obj, flat, elem, coef, add, rsrc, eptr, epts, partials, total;
};

AdjLayout adj_layout(const kw_sim *s, int n_steps) {
    AdjLayout L{};
    Carver cv;
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    for (int i = 0; i < 12; ++i) L.fld[i] = cv.take(N * sizeof(float));
    const size_t ns = s->src_flat.size();
    L.dJds = cv.take((size_t)std::max(1, n_steps) * std::max(1, s->cnt.n_elem) * sizeof(double));
    L.obj = cv.take(sizeof(double));
    L.flat = cv.take(std::max<size_t>(ns, 1) * sizeof(int));
    L.elem = cv.take(std::max<size_t>(ns, 1) * sizeof(int));
    L.coef = cv.take(std::max<size_t>(ns, 1) * sizeof(float));
    L.add = cv.take(std::max<size_t>(ns, 1) * sizeof(float));
    L.rsrc = cv.take(3 * std::max<size_t>(ns, 1) * sizeof(float));
    L.eptr = cv.take((size_t)(std::max(1, s->cnt.n_elem) + 1) * sizeof(int));
    L.epts = cv.take(std::max<size_t>(ns, 1) * sizeof(int));
    L.partials = cv.take((size_t)adj_objective_blocks(s->g) * sizeof(double));
    L.total = cv.off;
    return L;
}

// out[j] = IFT(m_j FT in[j]) for j < k, through the forward passes and the
// spectral scratch S1..S6 of the simulation (free between steps)
hipError_t spectral(kw_sim *s, int mode, float *const *in, float *const *out, int k) {
    hipStream_t st = s->stream;
    const GridDev &g = s->g;
    const LaunchCfg &c = s->cfg;
    const Tables &t = s->tab;
    float2 *sin[3] = {s->buf.S[1], s->buf.S[2], s->buf.S[3]};
    float2 *sout[3] = {s->buf.S[4], s->buf.S[5], s->buf.S[6]};
    hipError_t e;
    for (int j = 0; j < k; ++j)
        if ((e = launch_xfwd(st, g, c, t, in[j], sin[j])) != hipSuccess) return e;
    if ((e = launch_ypass(st, g, c, t, sin, k, false, nullptr, nullptr)) != hipSuccess) return e;
    if ((e = launch_zfused(st, g, c, t, mode, sin, sout)) != hipSuccess) return e;
    if ((e = launch_ypass(st, g, c, t, sout, k, true, nullptr, nullptr)) != hipSuccess) return e;
    for (int j = 0; j < k; ++j)
        if ((e = launch_xinv(st, g, c, t, sout[j], out[j], 1.0f)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace

size_t kw_adjoint_workspace_size(kw_sim *s, int32_t n_steps) {
    if (!s || n_steps < 1) {
        fail(KW_EINVAL, "sim is NULL or n_steps < 1");
        return 0;
    }
    return adj_layout(s, n_steps).total;
}

int kw_adjoint_create(kw_sim *s, const float *weights, int32_t n_steps, void *dev_workspace,
                      size_t ws_bytes, kw_adj **out) {
    if (!s || !weights || !dev_workspace || !out) return fail(KW_EINVAL, "NULL argument");
    *out = nullptr;
    if (n_steps < 1) return fail(KW_EINVAL, "n_steps must be >= 1");
    if (s->src_flat.empty()) return fail(KW_EINVAL, "the simulation has no source");
    if (s->src.kind != KW_SOURCE_MASS)
        return fail(KW_EINVAL, "the reverse mode covers mass sources only");
    const int n_window = n_steps - s->record_start + 1;
    if (n_window < 1)
        return fail(KW_EINVAL, "no recorded step: record_start %d > n_steps %d", s->record_start,
                    n_steps);
    const AdjLayout L = adj_layout(s, n_steps);
    if (ws_bytes < L.total)
        return fail(KW_ENOMEM, "adjoint workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    char *ws = reinterpret_cast<char *>(dev_workspace);
    kw_adj *adj = new kw_adj;
    adj->sim = s;
    adj->n_steps = n_steps;
    AdjDev &a = adj->a;
    auto F = [&](int i) { return reinterpret_cast<float *>(ws + L.fld[i]); };
    a.pb = F(0);
    for (int i = 0; i < 3; ++i) {
        a.ub[i] = F(1 + i);
        a.rb[i] = F(4 + i);
        a.d[i] = F(7 + i);
    }
    a.w = F(10);
    a.rbt = F(11);
    a.dJds = reinterpret_cast<double *>(ws + L.dJds);
    a.obj = reinterpret_cast<double *>(ws + L.obj);
    a.n_steps = n_steps;
    a.n_elem = s->cnt.n_elem;
    a.n_src = (int)s->src_flat.size();
    a.src_flat = reinterpret_cast<int *>(ws + L.flat);
    a.src_elem = reinterpret_cast<int *>(ws + L.elem);
    a.src_coef = reinterpret_cast<float *>(ws + L.coef);
    a.add = reinterpret_cast<float *>(ws + L.add);
    a.rsrc = reinterpret_cast<float *>(ws + L.rsrc);
    a.elem_ptr = reinterpret_cast<int *>(ws + L.eptr);
    a.elem_pts = reinterpret_cast<int *>(ws + L.epts);
    a.partials = reinterpret_cast<double *>(ws + L.partials);
    // the source points of each element, in increasing order (the fixed order
    // in which their shares of dJ/ds_e are summed)
    std::vector<int> eptr(a.n_elem + 1, 0), epts(s->src_flat.size());
    for (int e : s->src_elem) eptr[e + 1]++;
    for (int e = 0; e < a.n_elem; ++e) eptr[e + 1] += eptr[e];
    {
        std::vector<int> fill(eptr.begin(), eptr.end() - 1);
        for (size_t k = 0; k < s->src_elem.size(); ++k) epts[fill[s->src_elem[k]]++] = (int)k;
    }
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    hipStream_t st = s->stream;
    auto bail = [&](hipError_t e) {
        delete adj;
        return fail(KW_EDEVICE, "adjoint set-up: %s", hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(a.w, weights, N * sizeof(float), hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e);
    if ((e = launch_adj_weights(st, s->g, s->med, a.w, (float)(2.0 / n_window))) != hipSuccess)
        return bail(e);
    const size_t ns = s->src_flat.size();
    if ((e = hipMemcpyAsync(ws + L.flat, s->src_flat.data(), ns * sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ws + L.elem, s->src_elem.data(), ns * sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ws + L.coef, s->src_coef.data(), ns * sizeof(float), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ws + L.eptr, eptr.data(), eptr.size() * sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(ws + L.epts, epts.data(), ns * sizeof(int), hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e);
    for (int i = 0; i < 7; ++i)   // pb, ub, rb start at zero
        if ((e = launch_fill(st, F(i), N, 0.0f)) != hipSuccess) return bail(e);
    if ((e = hipMemsetAsync(a.dJds, 0, (size_t)n_steps * a.n_elem * sizeof(double), st)) != hipSuccess)
        return bail(e);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e);
    *out = adj;
    return KW_OK;
}

namespace {

// layout of a step record: du_x, du_y, du_z, rho_x, rho_y, rho_z, the packed
// spectrum of p (one N-float slot each, 256-byte aligned)
size_t record_slot(const kw_sim *s) {
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    return (N * sizeof(float) + 255) / 256 * 256;
}

// Reverse step n.  rec: a record of forward step n, or null when the
// simulation holds the state after step n (the forward divergence is then
// recomputed from u^(n+1/2)).
int reverse_step(kw_adj *adj, int n, const char *rec) {
    kw_sim *s = adj->sim;
    AdjDev a = adj->a;
    hipStream_t st = s->stream;
    const GridDev &g = s->g;
    const Medium &m = s->med;
    hipError_t e;
#define KW_A(call)                                                                  \
    do {                                                                            \
        if ((e = (call)) != hipSuccess)                                             \
            return fail(KW_EDEVICE, "adjoint step: %s", hipGetErrorString(e));      \
    } while (0)
    const float2 *p_spec;
    if (rec) {
        const size_t slot = record_slot(s);
        for (int i = 0; i < 3; ++i) {
            a.dfw[i] = reinterpret_cast<const float *>(rec + i * slot);
            a.rho[i] = reinterpret_cast<const float *>(rec + (3 + i) * slot);
        }
        p_spec = reinterpret_cast<const float2 *>(rec + 6 * slot);
    } else {
        // forward divergence of u^(n+1/2) (the nonlinear denominators need it)
        KW_A(spectral(s, ZM_DIV, s->buf.u, a.d, 3));
        for (int i = 0; i < 3; ++i) {
            a.dfw[i] = a.d[i];
            a.rho[i] = s->buf.rho[i];
        }
        p_spec = s->buf.S[0];
    }
    // x-row passes around the y and z passes of the transposed operators,
    // through the spectral scratch S1..S6 (S0, the pressure state, is left alone)
    const bool loss = n + 1 >= s->record_start;
    const LaunchCfg &c = s->cfg;
    const Tables &t = s->tab;
    float2 *const *S = s->buf.S;
    float2 *s12[2] = {S[1], S[2]}, *s45[2] = {S[4], S[5]};
    float2 *s123[3] = {S[1], S[2], S[3]}, *s456[3] = {S[4], S[5], S[6]};
    auto yzy = [&](int mode, float2 *const *in, float2 *const *out, int k) -> hipError_t {
        hipError_t r = launch_ypass(st, g, c, t, in, k, false, nullptr, nullptr);
        if (r == hipSuccess) r = launch_zfused(st, g, c, t, mode, in, out);
        if (r == hipSuccess) r = launch_ypass(st, g, c, t, out, k, true, nullptr, nullptr);
        return r;
    };
    KW_A(launch_adj_src(st, a, s->src, n));
    if (m.absorbing) {
        KW_A(launch_adjx(st, ADJX_EOS, g, c, t, m, s->src, a, p_spec, loss, nullptr, s12));
        KW_A(yzy(ZM_ABS, s12, s45, 2));
        KW_A(launch_adjx(st, ADJX_DEN_ABS, g, c, t, m, s->src, a, p_spec, loss, s45, s123));
    } else {
        KW_A(launch_adjx(st, ADJX_DEN, g, c, t, m, s->src, a, p_spec, loss, nullptr, s123));
    }
    KW_A(launch_adj_src_sum(st, a, n));
    KW_A(yzy(ZM_DIVT, s123, s456, 3));
    KW_A(launch_adjx(st, ADJX_VEL, g, c, t, m, s->src, a, nullptr, false, s456, s123));
    KW_A(yzy(ZM_GRADT, s123, s456, 3));
    KW_A(launch_adjx(st, ADJX_SUM, g, c, t, m, s->src, a, nullptr, false, s456, nullptr));
#undef KW_A
    return KW_OK;
}

}  // namespace

int kw_adjoint_step(kw_adj *adj, int32_t n) {
    if (!adj) return fail(KW_EINVAL, "adj is NULL");
    kw_sim *s = adj->sim;
    if (n < 0 || n >= adj->n_steps) return fail(KW_EINVAL, "step %d outside [0, %d)", n, adj->n_steps);
    if (s->steps != (long)n + 1)
        return fail(KW_ESTATE, "the simulation holds the state after step %ld, not %d", s->steps - 1, n);
    return reverse_step(adj, n, nullptr);
}

int64_t kw_adjoint_record_bytes(kw_adj *adj) {
    if (!adj) return -1;
    return (int64_t)(7 * record_slot(adj->sim));
}

int kw_adjoint_record(kw_adj *adj, void *dev_record, size_t bytes) {
    if (!adj || !dev_record) return fail(KW_EINVAL, "NULL argument");
    kw_sim *s = adj->sim;
    const size_t slot = record_slot(s);
    if (bytes < 7 * slot) return fail(KW_EINVAL, "record has %zu bytes, %zu needed", bytes, 7 * slot);
    char *r = reinterpret_cast<char *>(dev_record);
    for (int i = 0; i < 6; ++i) s->rec[i] = reinterpret_cast<float *>(r + i * slot);
    const hipError_t e = enqueue_step(s);
    for (int i = 0; i < 6; ++i) s->rec[i] = nullptr;
    if (e != hipSuccess) return fail(KW_EDEVICE, "kernel launch: %s", hipGetErrorString(e));
    const size_t N = (size_t)s->grid.nx * s->grid.ny * s->grid.nz;
    KW_HIP(hipMemcpyAsync(r + 6 * slot, s->buf.S[0], N * sizeof(float), hipMemcpyDeviceToDevice,
                          s->stream));
    s->steps += 1;
    s->stepped = true;
    return KW_OK;
}

int kw_adjoint_step_record(kw_adj *adj, int32_t n, const void *dev_record, size_t bytes) {
    if (!adj || !dev_record) return fail(KW_EINVAL, "NULL argument");
    if (n < 0 || n >= adj->n_steps) return fail(KW_EINVAL, "step %d outside [0, %d)", n, adj->n_steps);
    const size_t need = 7 * record_slot(adj->sim);
    if (bytes < need) return fail(KW_EINVAL, "record has %zu bytes, %zu needed", bytes, need);
    return reverse_step(adj, n, reinterpret_cast<const char *>(dev_record));
}

int kw_adjoint_objective(kw_adj *adj, double *J) {
    if (!adj || !J) return fail(KW_EINVAL, "NULL argument");
    kw_sim *s = adj->sim;
    if (!s->sen.all_points || !s->sen.p_sum2)
        return fail(KW_EINVAL, "the objective needs p_rms or intensity recorded at every point");
    if (s->steps != adj->n_steps)
        return fail(KW_ESTATE, "the simulation holds step %ld, the objective needs step %d",
                    s->steps, adj->n_steps);
    KW_HIP(launch_adj_objective(s->stream, s->g, adj->a.w, s->sen.p_sum2, adj->a.partials,
                                adj->a.obj));
    KW_HIP(hipMemcpyAsync(J, adj->a.obj, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    KW_HIP(hipStreamSynchronize(s->stream));
    return KW_OK;
}

int kw_adjoint_source_gradient(kw_adj *adj, double *dJds, size_t bytes) {
    if (!adj || !dJds) return fail(KW_EINVAL, "NULL argument");
    const size_t need = (size_t)adj->n_steps * adj->a.n_elem * sizeof(double);
    if (bytes < need) return fail(KW_EINVAL, "dst has %zu bytes, %zu needed", bytes, need);
    KW_HIP(hipMemcpyAsync(dJds, adj->a.dJds, need, hipMemcpyDeviceToHost, adj->sim->stream));
    KW_HIP(hipStreamSynchronize(adj->sim->stream));
    return KW_OK;
}

int kw_adjoint_gradient(kw_adj *adj, double *grad_amp, double *grad_phase) {
    if (!adj || !grad_amp || !grad_phase) return fail(KW_EINVAL, "NULL argument");
    kw_sim *s = adj->sim;
    if (s->src.signal) return fail(KW_EINVAL, "sampled drive signal: use kw_adjoint_source_gradient");
    const int ne = adj->a.n_elem, T = adj->n_steps;
    std::vector<double> d((size_t)T * ne);
    const int rc = kw_adjoint_source_gradient(adj, d.data(), d.size() * sizeof(double));
    if (rc != KW_OK) return rc;
    for (int e = 0; e < ne; ++e) {
        double ga = 0.0, gp = 0.0;
        for (int n = 0; n < T; ++n) {
            // s_e(n) = a_e sin(theta_n + phi_e), theta_n = omega (n + 1/2) dt
            const double th = s->src.omega_dt * ((double)n + 0.5) + s->src_phase[e];
            ga += d[(size_t)n * ne + e] * std::sin(th);
            gp += d[(size_t)n * ne + e] * s->src_amp[e] * std::cos(th);
        }
        grad_amp[e] = ga;
        grad_phase[e] = gp;
    }
    return KW_OK;
}

int kw_adjoint_destroy(kw_adj *adj) {
    if (!adj) return KW_OK;
    (void)hipStreamSynchronize(adj->sim->stream);
    delete adj;
    return KW_OK;
}

int kw_destroy(kw_sim *s) {
    if (!s) return KW_OK;
    (void)hipStreamSynchronize(s->stream);
    release(s);
    return KW_OK;
}

}  // extern "C"
