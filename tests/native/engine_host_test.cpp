// Host test of the engine's set-up and error paths, linked against the host
// stand-in of the HIP runtime (hip_host_stub.cpp) and built with
// AddressSanitizer or ThreadSanitizer.
//   threads: kw_prepare / kw_create_prepared / kw_create from 8 threads at
//            once; every workspace must hold the same bytes as a serial run
//   errors:  statuses of failed device calls reach the caller unchanged
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "kw.h"

extern "C" {
extern std::atomic<int> kw_stub_fail_launches;
}

namespace {

struct Inputs {
    kw_grid grid{};
    kw_medium medium{};
    kw_source source{};
    kw_sensor sensor{};
    std::vector<float> c0, rho0, alpha0, bona, amp, phase;
    std::vector<int64_t> src_idx, sen_idx;
    std::vector<int32_t> elem;
    size_t npts = 0;
};

// 0: heterogeneous nonlinear absorbing, mass source of 3 elements, mask sensor
//    with series, harmonics and velocity series;
// 1: homogeneous absorbing (merged absorption), force source, all-point sensors;
// 2: 2/3/5 lengths, lossless nonlinear, pressure source, mask sensor.
void make_inputs(int variant, Inputs &in) {
    const int dims[3][3] = {{48, 40, 36}, {32, 32, 32}, {30, 45, 50}};
    kw_grid &g = in.grid;
    g.nx = dims[variant][0];
    g.ny = dims[variant][1];
    g.nz = dims[variant][2];
    g.dx = g.dy = g.dz = 1e-4;
    g.cfl = 0.3;
    for (int a = 0; a < 3; ++a) {
        g.pml_size[a] = 4;
        g.pml_alpha[a] = 2.0;
    }
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    in.npts = N;
    std::mt19937 rng(1234 + variant);
    std::uniform_real_distribution<float> u01(0.0f, 1.0f);
    kw_medium &m = in.medium;
    m.alpha_power = 1.5;
    if (variant == 0) {
        in.c0.resize(N);
        in.rho0.resize(N);
        in.alpha0.resize(N);
        in.bona.resize(N);
        for (size_t i = 0; i < N; ++i) {
            in.c0[i] = 1450.0f + 200.0f * u01(rng);
            in.rho0[i] = 950.0f + 150.0f * u01(rng);
            in.alpha0[i] = 0.5f + u01(rng);
            in.bona[i] = 5.0f + 4.0f * u01(rng);
        }
        m.c0 = in.c0.data();
        m.rho0 = in.rho0.data();
        m.alpha0 = in.alpha0.data();
        m.bona = in.bona.data();
        m.flags = KW_NONLINEAR | KW_ABSORBING;
    } else {
        m.c0_scalar = 1500.0;
        m.rho0_scalar = 1000.0;
        m.alpha0_scalar = 0.75;
        m.bona_scalar = 5.0;
        m.flags = variant == 1 ? (KW_NONLINEAR | KW_ABSORBING) : KW_NONLINEAR;
    }
    // source: every 7th point of plane z = 5, three elements
    const int ne = 3;
    for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; x += 7) {
            in.src_idx.push_back(x + (int64_t)g.nx * (y + (int64_t)g.ny * 5));
            in.elem.push_back((x + y) % ne);
        }
    in.amp = {1e5f, 2e5f, 3e5f};
    in.phase = {0.0f, 0.5f, 1.0f};
    kw_source &s = in.source;
    s.n_points = (int64_t)in.src_idx.size();
    s.index = in.src_idx.data();
    s.element = in.elem.data();
    s.n_elements = ne;
    s.amp = in.amp.data();
    s.phase = in.phase.data();
    s.freq = 1e6;
    s.kind = variant == 0 ? KW_SOURCE_MASS : variant == 1 ? KW_SOURCE_FORCE : KW_SOURCE_PRESSURE;
    s.axis = 2;
    kw_sensor &z = in.sensor;
    z.record_start = 2;
    if (variant == 1) {
        z.record = KW_REC_P_MAX | KW_REC_P_RMS;
    } else {
        for (size_t i = 11; i < N; i += 997) in.sen_idx.push_back((int64_t)i);
        z.n_points = (int64_t)in.sen_idx.size();
        z.index = in.sen_idx.data();
        z.record = KW_REC_P_MAX | KW_REC_P_SERIES | KW_REC_P_MIN;
        if (variant == 0) z.record |= KW_REC_HARMONICS | KW_REC_U_SERIES | KW_REC_INTENSITY;
        z.series_capacity = 16;
        z.n_harmonics = 3;
    }
}

struct Buffer {
    unsigned char *p = nullptr;
    size_t n = 0;
    explicit Buffer(size_t bytes) : n(bytes) {
        p = static_cast<unsigned char *>(std::aligned_alloc(256, (bytes + 255) / 256 * 256));
        std::memset(p, 0xAB, n);
    }
    ~Buffer() { std::free(p); }
};

// Set one simulation up on a host "workspace" and return its bytes.
int set_up(const Inputs &in, bool split, std::vector<unsigned char> &out) {
    const size_t need = kw_workspace_size(&in.grid, &in.medium, &in.source, &in.sensor);
    if (need == 0) return -100;
    Buffer ws(need);
    kw_sim *sim = nullptr;
    int rc;
    if (split) {
        kw_plan *plan = nullptr;
        rc = kw_prepare(&in.grid, &in.medium, &in.source, &in.sensor, &plan);
        if (rc != KW_OK) return rc;
        if (kw_plan_workspace_size(plan) != need) {
            kw_plan_destroy(plan);
            return -101;
        }
        rc = kw_create_prepared(plan, ws.p, ws.n, nullptr, &sim);
        kw_plan_destroy(plan);
    } else {
        rc = kw_create(&in.grid, &in.medium, &in.source, &in.sensor, ws.p, ws.n, nullptr, &sim);
    }
    if (rc != KW_OK) return rc;
    out.assign(ws.p, ws.p + ws.n);
    return kw_destroy(sim);
}

int run_threads() {
    int bad = 0;
    for (int variant = 0; variant < 3; ++variant) {
        Inputs in;
        make_inputs(variant, in);
        std::vector<unsigned char> ref;
        int rc = set_up(in, false, ref);
        if (rc != KW_OK) {
            std::printf("variant %d: serial set-up failed (%d): %s\n", variant, rc, kw_last_error());
            return 1;
        }
        std::atomic<int> mismatches{0}, failures{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < 8; ++t) {
            pool.emplace_back([&, t] {
                for (int rep = 0; rep < 3; ++rep) {
                    std::vector<unsigned char> got;
                    const int r = set_up(in, (t + rep) % 2 == 0, got);
                    if (r != KW_OK) failures++;
                    else if (got != ref) mismatches++;
                }
            });
        }
        for (auto &th : pool) th.join();
        std::printf("variant %d: %zu workspace bytes, 24 concurrent set-ups, %d failures, %d mismatches\n",
                    variant, ref.size(), failures.load(), mismatches.load());
        bad += failures.load() + mismatches.load();
    }
    return bad ? 1 : 0;
}

#define EXPECT(cond, ...)                        \
    do {                                         \
        if (!(cond)) {                           \
            std::printf("FAILED: " __VA_ARGS__); \
            std::printf("\n");                   \
            return 1;                            \
        }                                        \
    } while (0)

int run_errors() {
    Inputs in;
    make_inputs(0, in);
    const size_t need = kw_workspace_size(&in.grid, &in.medium, &in.source, &in.sensor);
    Buffer ws(need);
    kw_sim *sim = nullptr;
    EXPECT(kw_create(&in.grid, &in.medium, &in.source, &in.sensor, ws.p, ws.n, nullptr, &sim) == KW_OK,
           "create: %s", kw_last_error());
    std::vector<float> dst(in.npts);
    EXPECT(kw_gather_field(sim, KW_FIELD_P, dst.data(), 0) == KW_OK, "gather_field P ok path");
    kw_stub_fail_launches = 1;
    int rc = kw_gather_field(sim, KW_FIELD_P, dst.data(), 0);
    EXPECT(rc == KW_EDEVICE, "gather_field P with a failing transform returned %d", rc);
    rc = kw_gather(sim, KW_REC_P_FINAL, dst.data(), dst.size() * sizeof(float), 0);
    EXPECT(rc == KW_EDEVICE, "gather P_FINAL with a failing transform returned %d", rc);
    rc = kw_gather_field(sim, KW_FIELD_UX, dst.data(), 0);
    EXPECT(rc == KW_EDEVICE, "gather_field u_x with a failing copy returned %d", rc);
    rc = kw_step(sim, 1);
    EXPECT(rc == KW_EDEVICE, "step with failing launches returned %d", rc);
    kw_stub_fail_launches = 0;
    EXPECT(kw_destroy(sim) == KW_OK, "destroy");

    kw_sim *s2 = nullptr;
    EXPECT(kw_create_prepared(nullptr, ws.p, ws.n, nullptr, &s2) == KW_EINVAL && !s2, "null plan");
    kw_plan *plan = nullptr;
    EXPECT(kw_prepare(&in.grid, &in.medium, &in.source, &in.sensor, &plan) == KW_OK, "prepare");
    EXPECT(kw_create_prepared(plan, ws.p + 16, ws.n - 16, nullptr, &s2) == KW_EINVAL && !s2,
           "misaligned workspace");
    EXPECT(kw_create_prepared(plan, ws.p, need - 1, nullptr, &s2) == KW_ENOMEM && !s2,
           "small workspace");
    kw_stub_fail_launches = 1;
    rc = kw_create_prepared(plan, ws.p, ws.n, nullptr, &s2);
    kw_stub_fail_launches = 0;
    EXPECT(rc == KW_EDEVICE && !s2, "create_prepared with failing uploads returned %d", rc);
    EXPECT(kw_plan_destroy(plan) == KW_OK && kw_plan_destroy(nullptr) == KW_OK, "plan destroy");
    EXPECT(kw_plan_workspace_size(nullptr) == 0, "plan size of NULL");
    kw_grid bad = in.grid;
    bad.nx = 7;
    plan = reinterpret_cast<kw_plan *>(0x1);
    EXPECT(kw_prepare(&bad, &in.medium, &in.source, &in.sensor, &plan) == KW_EUNSUPPORTED && !plan,
           "prepare of an odd nx");
    // kw_create_static: the workspace ends before the six spectral arrays,
    // which must fit the static array (1 MiB in the host stand-in)
    {
        Inputs sm;
        make_inputs(1, sm);
        sm.grid.nx = sm.grid.ny = sm.grid.nz = 16;
        for (int a = 0; a < 3; ++a) sm.grid.pml_size[a] = 2;
        sm.source.n_points = 0;
        const size_t full = kw_workspace_size(&sm.grid, &sm.medium, &sm.source, &sm.sensor);
        const size_t spec = (4 * 16 * 16 * 16 + 255) / 256 * 256;
        Buffer w2(full - 6 * spec);
        kw_sim *st = nullptr;
        EXPECT(kw_create_static(&sm.grid, &sm.medium, &sm.source, &sm.sensor, w2.p, w2.n - 1,
                                nullptr, &st) == KW_ENOMEM && !st, "static: one byte short");
        rc = kw_create_static(&sm.grid, &sm.medium, &sm.source, &sm.sensor, w2.p, w2.n, nullptr, &st);
        EXPECT(rc == KW_OK && st, "static create returned %d: %s", rc, kw_last_error());
        kw_stats_t stt;
        EXPECT(kw_stats(st, &stt) == KW_OK && (size_t)stt.workspace_bytes == full - 6 * spec,
               "static workspace bytes");
        EXPECT(kw_destroy(st) == KW_OK, "static destroy");
        // 48 x 40 x 36: six spectra of 276480 bytes exceed the static array
        Buffer w3(need);
        st = nullptr;
        rc = kw_create_static(&in.grid, &in.medium, &in.source, &in.sensor, w3.p, w3.n, nullptr, &st);
        EXPECT(rc == KW_EUNSUPPORTED && !st, "static create of a grid too large returned %d", rc);
    }
    // reverse mode with step records: argument checks, the step a record
    // advances, and failed launches reported as such
    {
        kw_sim *sm = nullptr;
        Buffer w4(need);
        EXPECT(kw_create(&in.grid, &in.medium, &in.source, &in.sensor, w4.p, w4.n, nullptr, &sm) == KW_OK,
               "create for the adjoint: %s", kw_last_error());
        const int T = 4;
        const size_t anb = kw_adjoint_workspace_size(sm, T);
        EXPECT(anb > 0, "adjoint workspace size");
        Buffer aw(anb);
        std::vector<float> weights(in.npts, 1.0f);
        kw_adj *adj = nullptr;
        EXPECT(kw_adjoint_create(sm, weights.data(), T, aw.p, aw.n, &adj) == KW_OK && adj,
               "adjoint create: %s", kw_last_error());
        const int64_t rb = kw_adjoint_record_bytes(adj);
        EXPECT(rb >= (int64_t)(7 * in.npts * sizeof(float)) && kw_adjoint_record_bytes(nullptr) == -1,
               "record bytes %lld", (long long)rb);
        Buffer rec((size_t)rb);
        EXPECT(kw_adjoint_record(adj, nullptr, rec.n) == KW_EINVAL, "record into NULL");
        EXPECT(kw_adjoint_record(adj, rec.p, rec.n - 1) == KW_EINVAL, "record one byte short");
        kw_stats_t st0, st1;
        EXPECT(kw_stats(sm, &st0) == KW_OK, "stats");
        EXPECT(kw_adjoint_record(adj, rec.p, rec.n) == KW_OK, "record: %s", kw_last_error());
        EXPECT(kw_stats(sm, &st1) == KW_OK && st1.steps == st0.steps + 1, "a record advances one step");
        EXPECT(kw_adjoint_step_record(adj, T, rec.p, rec.n) == KW_EINVAL, "reverse step out of range");
        EXPECT(kw_adjoint_step_record(adj, 0, rec.p, rec.n - 1) == KW_EINVAL, "reverse step, short record");
        EXPECT(kw_adjoint_step_record(adj, 0, nullptr, rec.n) == KW_EINVAL, "reverse step, NULL record");
        EXPECT(kw_adjoint_step_record(adj, 0, rec.p, rec.n) == KW_OK, "reverse step: %s", kw_last_error());
        kw_stub_fail_launches = 1;
        rc = kw_adjoint_record(adj, rec.p, rec.n);
        EXPECT(rc == KW_EDEVICE, "record with failing launches returned %d", rc);
        rc = kw_adjoint_step_record(adj, 0, rec.p, rec.n);
        EXPECT(rc == KW_EDEVICE, "reverse step with failing launches returned %d", rc);
        kw_stub_fail_launches = 0;
        EXPECT(kw_step(sm, 1) == KW_OK, "step after a failed record");
        EXPECT(kw_adjoint_destroy(adj) == KW_OK && kw_destroy(sm) == KW_OK, "adjoint destroy");
    }
    std::printf("error paths ok\n");
    return 0;
}

// kw_set_plan: schedules for each kind of FFT engine instantiation are
// accepted (fixed widths 8, 16 and 32, the radix sets {8}, {16}, {8, 4},
// {6, 4}, the 12- and 20-wide engines, the generic fallback of a radix-32
// schedule with other radices), schedules that are not a factorisation of the
// length are refused, and a step runs afterwards
int run_plans() {
    struct Case { int variant, axis; std::vector<int32_t> rad; int want; };
    const Case cases[] = {
        {1, 2, {32}, KW_OK},          {1, 2, {8, 4}, KW_OK},      {1, 2, {16, 2}, KW_OK},
        {1, 1, {4, 4, 2}, KW_OK},     {1, 0, {16}, KW_OK},        {1, 0, {8, 2}, KW_OK},
        {1, 2, {8, 8}, KW_EINVAL},    {1, 1, {3, 11}, KW_EINVAL},
        {0, 2, {6, 6}, KW_OK},        {0, 0, {6, 4}, KW_OK},      {0, 1, {10, 4}, KW_OK},
        {0, 2, {12, 3}, KW_OK},       {0, 0, {24}, KW_OK},        {0, 2, {5, 7}, KW_EINVAL},
        {2, 2, {10, 5}, KW_OK},       {2, 1, {15, 3}, KW_OK},       {2, 1, {5, 9}, KW_EINVAL},
    };
    for (const Case &c : cases) {
        Inputs in;
        make_inputs(c.variant, in);
        Buffer ws(kw_workspace_size(&in.grid, &in.medium, &in.source, &in.sensor));
        kw_sim *sim = nullptr;
        EXPECT(kw_create(&in.grid, &in.medium, &in.source, &in.sensor, ws.p, ws.n, nullptr, &sim) == KW_OK,
               "create: %s", kw_last_error());
        const int rc = kw_set_plan(sim, c.axis, c.rad.data(), (int32_t)c.rad.size(), 0);
        EXPECT(rc == c.want, "variant %d axis %d: set_plan returned %d, expected %d (%s)", c.variant,
               c.axis, rc, c.want, kw_last_error());
        EXPECT(kw_step(sim, 1) == KW_OK, "step after set_plan: %s", kw_last_error());
        EXPECT(kw_destroy(sim) == KW_OK, "destroy");
    }
    // a 32-wide schedule with a smaller radix runs on the generic engine
    {
        Inputs in;
        make_inputs(1, in);
        in.grid.nz = 64;
        in.npts = (size_t)in.grid.nx * in.grid.ny * in.grid.nz;
        Buffer ws(kw_workspace_size(&in.grid, &in.medium, &in.source, &in.sensor));
        kw_sim *sim = nullptr;
        EXPECT(kw_create(&in.grid, &in.medium, &in.source, &in.sensor, ws.p, ws.n, nullptr, &sim) == KW_OK,
               "create 32x32x64: %s", kw_last_error());
        const int32_t r[2] = {32, 2};
        EXPECT(kw_set_plan(sim, 2, r, 2, 0) == KW_OK, "schedule 32.2: %s", kw_last_error());
        EXPECT(kw_step(sim, 1) == KW_OK, "step");
        EXPECT(kw_destroy(sim) == KW_OK, "destroy");
    }
    std::printf("plans ok\n");
    return 0;
}

}  // namespace

int main(int argc, char **argv) {
    const char *mode = argc > 1 ? argv[1] : "threads";
    if (!std::strcmp(mode, "threads")) return run_threads();
    if (!std::strcmp(mode, "errors")) return run_errors();
    if (!std::strcmp(mode, "plans")) return run_plans();
    std::printf("unknown mode %s\n", mode);
    return 2;
}
