// Launchers of the x-pass kernels (all FFT engines).
#include "kernels_impl.h"

namespace kw {

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
    return x_lds_bytes(g.M, g.nx, c.tb_x, line);
}
#define KW_XLAUNCH(KERNEL, LINE) KW_XLAUNCH_N(KERNEL, LINE, 1)
#define KW_XLAUNCH_N(KERNEL, LINE, NY)                                               \
    do {                                                                             \
        dim3 grid((g.rows + c.tb_x - 1) / c.tb_x, NY);                               \
        dim3 block(c.tb_x * c.px.L);                                                 \
        size_t lds = x_lds(g, c, LINE);                                              \
        KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((KERNEL<Eng>), grid, block, lds, s, a)); \
    } while (0)

hipError_t launch_xvel(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, float2 *const *S, float *const *u,
                       const SourceDev &src, const SensorDev &sen, const Counters &cnt) {
    XArgs a = make_xargs(g, c, t);
    a.m = m;
    a.src = src;
    a.sen = sen;
    a.cnt = cnt;
    for (int i = 0; i < 3; ++i) {
        a.Sin[i] = S[i];
        a.Sout[i] = S[i];
        a.fld[i] = u[i];
    }
    dim3 grid((g.rows + c.tb_x - 1) / c.tb_x, 3);
    dim3 block(c.tb_x * c.px.L);
    const int fl = (sen.u_series ? XV_USER : 0) |
                   (src.row_ptr && src.kind == KW_SOURCE_FORCE ? XV_FORCE : 0);
    const size_t lds = x_lds(g, c, fl != 0);
    switch (fl) {
    case 0: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xvel<Eng, 0>), grid, block, lds, s, a)); break;
    case 1: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xvel<Eng, 1>), grid, block, lds, s, a)); break;
    case 2: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xvel<Eng, 2>), grid, block, lds, s, a)); break;
    default: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xvel<Eng, 3>), grid, block, lds, s, a)); break;
    }
    return hipGetLastError();
}

hipError_t launch_xden(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, const SourceDev &src, const SensorDev &sen,
                       const Counters &cnt, float2 *const *Sin, float *const *rho,
                       float *rho_total, float2 *const *Sout, bool rho0_sum_in_z,
                       float *const *rec) {
    XArgs a = make_xargs(g, c, t);
    a.rho0_sum_in_z = rho0_sum_in_z ? 1 : 0;
    if (rec) {
        for (int i = 0; i < 3; ++i) {
            a.rec_d[i] = rec[i];
            a.rec_rho[i] = rec[3 + i];
        }
    }
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
    if (!eng_fixed(c.eng_x) || eng_general(c.eng_x) == ENG_F12 || eng_wide(c.eng_x)) {
        // generic and mixed-radix engines: three thread groups per row (see
        // kw_xden3; their wider register arrays leave no room for the sums)
        a.tb = c.tb_den;
        dim3 grid((g.rows + c.tb_den - 1) / c.tb_den);
        dim3 block(3 * c.tb_den * c.px.L);
        const size_t lds = den_lds_bytes(g.M, g.nx, c.tb_den, den_needs_line(m, src, sen));
#define KW_DEN3(ENGT)                                                                              \
    do {                                                                                           \
        if (m.absorbing) hipLaunchKernelGGL((kw_xden3<ENGT, true>), grid, block, lds, s, a);       \
        else hipLaunchKernelGGL((kw_xden3<ENGT, false>), grid, block, lds, s, a);                  \
    } while (0)
        if (c.eng_x == ENG_G16) KW_DEN3(EngGeneric<16>);
        else if (c.eng_x == ENG_F12) KW_DEN3(EngFixed<12>);
        else if (c.eng_x == ENG_F12_64) KW_DEN3(EngFixed12_64);
        else if (c.eng_x == ENG_F20) KW_DEN3(EngFixed<20>);
        else if (c.eng_x == ENG_F32) KW_DEN3(EngFixed<32>);
        else KW_DEN3(EngGeneric<32>);
#undef KW_DEN3
        return hipGetLastError();
    }
    dim3 grid((g.rows + c.tb_x - 1) / c.tb_x);
    dim3 block(c.tb_x * c.px.L);
    // source values and sensor lines use the FFT buffers (2 M + 2 floats a
    // row); the line holds the row's rho0 values of a rho0 map
    const size_t lds = x_lds(g, c, m.rho0.map != nullptr);
    const int variant = (m.absorbing ? 1 : 0) | (src.row_ptr && src.kind == KW_SOURCE_MASS ? 2 : 0);
    // fixed engines only (the generic ones took the branch above)
#define KW_DEN1(ENGT)                                                                              \
    do {                                                                                           \
        switch (variant) {                                                                         \
        case 0: hipLaunchKernelGGL((kw_xden<ENGT, false, false>), grid, block, lds, s, a); break;  \
        case 1: hipLaunchKernelGGL((kw_xden<ENGT, true, false>), grid, block, lds, s, a); break;   \
        case 2: hipLaunchKernelGGL((kw_xden<ENGT, false, true>), grid, block, lds, s, a); break;   \
        default: hipLaunchKernelGGL((kw_xden<ENGT, true, true>), grid, block, lds, s, a); break;   \
        }                                                                                          \
    } while (0)
    if (c.eng_x == ENG_F4) KW_DEN1(EngFixed<4>);
    else if (c.eng_x == ENG_F8) KW_DEN1(EngFixed<8>);
    else if (c.eng_x == ENG_F8P) KW_DEN1(EngFixed8P);
    else if (c.eng_x == ENG_F8_84) KW_DEN1(EngFixed8_84);
    else if (c.eng_x == ENG_F16P) KW_DEN1(EngFixed16P);
    else KW_DEN1(EngFixed<16>);
#undef KW_DEN1
    return hipGetLastError();
}

hipError_t launch_xeos(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                       const Medium &m, const SourceDev &src, const SensorDev &sen,
                       const Counters &cnt, float2 *const *Sin, const float *rho_total,
                       float2 *Sout, bool merged) {
    XArgs a = make_xargs(g, c, t);
    a.m = m;
    a.src = src;
    a.sen = sen;
    a.cnt = cnt;
    a.Sin[0] = Sin[0];
    a.Sin[1] = Sin[1];
    a.rho_total = const_cast<float *>(rho_total);
    a.Sout[0] = Sout;
    // mask sensor points and pressure-source values are picked out of a row
    // through a line that aliases the row's FFT buffer (no LDS of its own)
    const bool mask = sen.row_ptr != nullptr && !sen.all_points;
    const bool psrc = src.row_ptr != nullptr && src.kind == KW_SOURCE_PRESSURE;
    const bool extra = sen.p_min != nullptr || sen.harm != nullptr || psrc;
    dim3 grid((g.rows + c.tb_x - 1) / c.tb_x);
    dim3 block(c.tb_x * c.px.L);
    const size_t lds = x_lds(g, c, false);
    const int variant = (mask || extra ? 1 : 0) | (merged ? 2 : 0);
    switch (variant) {
    case 0: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xeos<Eng, false, false>), grid, block, lds, s, a)); break;
    case 1: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xeos<Eng, true, false>), grid, block, lds, s, a)); break;
    case 2: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xeos<Eng, false, true>), grid, block, lds, s, a)); break;
    default: KW_ENGINE_SWITCH(c.eng_x, hipLaunchKernelGGL((kw_xeos<Eng, true, true>), grid, block, lds, s, a)); break;
    }
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

}  // namespace kw
