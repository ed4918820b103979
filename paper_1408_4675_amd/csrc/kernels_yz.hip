// Launchers of the y-pass and fused z-pass kernels (all FFT engines).
#include "kernels_impl.h"

namespace kw {

hipError_t launch_ypass(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                        float2 *const *fields, int nfields, bool inverse,
                        const Counters *prologue, const SourceDev *src, const SensorDev *sen,
                        float2 *const *dst) {
    YArgs a{};
    for (int i = 0; i < nfields; ++i) {
        a.f[i] = fields[i];
        a.o[i] = dst ? dst[i] : fields[i];
    }
    a.M = g.M;
    a.ny = g.ny;
    a.plan = inverse ? c.pyi : c.py;
    a.tw = t.tw_y;
    a.tb = c.tb_y;
    a.prologue = prologue != nullptr;
    if (prologue) a.cnt = *prologue;
    if (src) a.src = *src;
    if (sen && sen->harm) {
        a.hw = sen->hw;
        a.n_harm = sen->n_harm;
        a.harm_wdt = sen->harm_wdt;
    }
    a.ntiles = (g.M + a.tb - 1) / a.tb;
    a.nz = g.nz;
    // one workgroup per (tile, z plane) in XCD-aware order (xcd_order), per field
    dim3 grid(xcd_grid(a.ntiles * g.nz, line_group(a.tb), 1), 1, nfields);
    dim3 block(a.tb * a.plan.L);
    size_t lds = col_lds_bytes(g.ny, a.tb);
    if (block.x > 512) {
        // wide tiles: 1024-thread instantiations of the fixed engines
        if (c.eng_y == ENG_F16) {
            if (inverse) hipLaunchKernelGGL((kw_ypass<EngFixed<16>, true, 1024>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((kw_ypass<EngFixed<16>, false, 1024>), grid, block, lds, s, a);
        } else if (c.eng_y == ENG_F16P) {
            if (inverse) hipLaunchKernelGGL((kw_ypass<EngFixed16P, true, 1024>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((kw_ypass<EngFixed16P, false, 1024>), grid, block, lds, s, a);
        } else if (c.eng_y == ENG_F8P) {
            if (inverse) hipLaunchKernelGGL((kw_ypass<EngFixed8P, true, 1024>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((kw_ypass<EngFixed8P, false, 1024>), grid, block, lds, s, a);
        } else if (c.eng_y == ENG_F8_84) {
            if (inverse) hipLaunchKernelGGL((kw_ypass<EngFixed8_84, true, 1024>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((kw_ypass<EngFixed8_84, false, 1024>), grid, block, lds, s, a);
        } else if (c.eng_y == ENG_F8) {
            if (inverse) hipLaunchKernelGGL((kw_ypass<EngFixed<8>, true, 1024>), grid, block, lds, s, a);
            else hipLaunchKernelGGL((kw_ypass<EngFixed<8>, false, 1024>), grid, block, lds, s, a);
        } else {
            return hipErrorInvalidConfiguration;
        }
        return hipGetLastError();
    }
    KW_ENGINE_SWITCH(c.eng_y, {
        if (inverse) hipLaunchKernelGGL((kw_ypass<Eng, true>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((kw_ypass<Eng, false>), grid, block, lds, s, a);
    });
    return hipGetLastError();
}

static int z_inputs(int mode) {
    return (mode == ZM_GRAD) ? 1 : (mode == ZM_ABS || mode == ZM_ABSM) ? 2 : 3;
}
static int z_outputs(int mode) { return (mode == ZM_ABS) ? 2 : (mode == ZM_ABSM) ? 1 : 3; }

static ZArgs make_zargs(const GridDev &g, const LaunchCfg &c, const Tables &t, int mode,
                        float2 *const *in, float2 *const *out) {
    ZArgs a{};
    const int nin = z_inputs(mode);
    const int nout = z_outputs(mode);
    for (int i = 0; i < nin; ++i) a.in[i] = in[i];
    for (int i = 0; i < nout; ++i) a.out[i] = out[i];
    a.g = g;
    a.t = t;
    a.pf = c.pz;
    a.pi = c.pzi;
    a.tb = c.tb_z;
    a.ntiles = (g.M + a.tb - 1) / a.tb;
    return a;
}

hipError_t launch_zfused(hipStream_t s, const GridDev &g, const LaunchCfg &c, const Tables &t,
                         int mode, float2 *const *in, float2 *const *out, float sa, float sb,
                         float2 *const *add0) {
    ZArgs a = make_zargs(g, c, t, mode, in, out);
    a.sa = sa;
    a.sb = sb;
    if (add0 && (mode == ZM_ABS || mode == ZM_ABSM)) {
        a.add0[0] = add0[0];
        a.add0[1] = add0[1];
    }
    int eng = c.eng_z;
    if (mode == ZM_ABSM) {
        // the merged absorption's own engine and plans (see LaunchCfg)
        eng = c.eng_za;
        a.pf = c.pza;
        a.pi = c.pzai;
        a.tb = c.tb_za;
        a.ntiles = (g.M + a.tb - 1) / a.tb;
    }
    const bool fixed_z = eng_fixed(eng);
    if (mode == ZM_ABSM && a.tb * a.pf.L > 512 && a.tb > 1) {
        // the merged absorption holds two spectra per thread: they do not fit
        // the registers of a 1024-thread block, so it runs half-width tiles
        a.tb /= 2;
        a.ntiles = (g.M + a.tb - 1) / a.tb;
    }
    // The gradient of a fixed engine keeps the forward spectrum for its three
    // outputs in one block.  The kept spectrum does not fit blocks of 512
    // threads or more (one block per CU), so on long columns the gradient runs
    // narrower tiles (1024 points: 4 columns, 256 threads) rather than one
    // block per output, which re-reads the input and transforms it three times
    // (measured at 1024^3: 9.8 ms against 11.0 ms).  The generic and the
    // 20- and 32-wide engines run one block per output (split).
    if (mode == ZM_GRAD && fixed_z && !eng_wide(eng)) {
        while (a.tb > 1 && a.tb * a.pf.L >= 512) a.tb /= 2;
        a.ntiles = (g.M + a.tb - 1) / a.tb;
    }
    const bool split = mode == ZM_GRAD && (!fixed_z || eng_wide(eng) || a.tb * a.pf.L >= 512);
    // one block per tile and output, in XCD-aware order (xcd_order): the
    // gradient's blocks (one, or three when split) in a 1D grid, the other
    // modes' outputs along blockIdx.y
    const int nblk = a.ntiles * g.ny;
    const int G = line_group(a.tb);
    dim3 grid;
    if (mode == ZM_GRAD) grid = dim3(xcd_grid(nblk, G, split ? 3 : 1), 1);
    else grid = dim3(xcd_grid(nblk, G, 1), z_outputs(mode));
    dim3 block(a.tb * a.pf.L);
    size_t lds = zcol_lds_bytes(g.nz, a.tb);
#define KW_ZMODES(ENGT, MAXT)                                                                  \
    do {                                                                                       \
        if (mode == ZM_GRAD && split) hipLaunchKernelGGL((kw_zfused<ENGT, ZM_GRAD, MAXT, true>), grid, block, lds, s, a); \
        else if (mode == ZM_GRAD) hipLaunchKernelGGL((kw_zfused<ENGT, ZM_GRAD, MAXT>), grid, block, lds, s, a);   \
        else if (mode == ZM_DIV) hipLaunchKernelGGL((kw_zfused<ENGT, ZM_DIV, MAXT>), grid, block, lds, s, a); \
        else if (mode == ZM_ABS) hipLaunchKernelGGL((kw_zfused<ENGT, ZM_ABS, MAXT>), grid, block, lds, s, a); \
        else if (mode == ZM_DIVT) hipLaunchKernelGGL((kw_zfused<ENGT, ZM_DIVT, MAXT>), grid, block, lds, s, a); \
        else if (mode == ZM_ABSM) hipLaunchKernelGGL((kw_zfused<ENGT, ZM_ABSM, MAXT>), grid, block, lds, s, a); \
        else hipLaunchKernelGGL((kw_zfused<ENGT, ZM_GRADT, MAXT>), grid, block, lds, s, a);    \
    } while (0)
    if (block.x > 512) {
        // wide tiles: 1024-thread instantiations of the fixed engines
        if (eng == ENG_F16) KW_ZMODES(EngFixed<16>, 1024);
        else if (eng == ENG_F16P) KW_ZMODES(EngFixed16P, 1024);
        else if (eng == ENG_F8P) KW_ZMODES(EngFixed8P, 1024);
        else if (eng == ENG_F8_84) KW_ZMODES(EngFixed8_84, 1024);
        else if (eng == ENG_F8) KW_ZMODES(EngFixed<8>, 1024);
        else return hipErrorInvalidConfiguration;
        return hipGetLastError();
    }
    KW_ENGINE_SWITCH(eng, KW_ZMODES(Eng, 512));
#undef KW_ZMODES
    return hipGetLastError();
}

}  // namespace kw
