"""GPU (HIP, float32) versus the FP64 CPU oracle, through the C ABI.

Tolerances: rel L2 <= 1e-4 per recorded field for linear lossless runs and
<= 1e-3 for nonlinear or absorbing runs; exact-solution checks at 1e-4.
"""
import numpy as np
import pytest

from oracle import Oracle
from paper_1408_4675_amd import scenarios as sc
from tests._parity import compare_outputs, rel_l2

pytestmark = pytest.mark.gpu

REPORT = []


@pytest.fixture(scope="module")
def kw():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4675_amd import _abi as A
    from paper_1408_4675_amd.simulation import Simulation
    A.load()
    return A, Simulation


def _banner(name):
    print("\n[case] %s" % name, flush=True)


def _run_both(kw, scen, steps, graph_steps=None, plans=()):
    A, Simulation = kw
    _banner("%s steps=%d plans %s" % (scen.name, steps, list(plans)))
    sim = Simulation(scen, graph_steps=graph_steps)
    for axis, rad in plans:
        sim.set_plan(axis, rad)
    sim.step(steps)
    orc = Oracle(scen)
    orc.step(steps)
    return sim, orc


# ---------------------------------------------------------------------------
# transform-level checks
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(48, 20, 18), (64, 64, 64), (40, 45, 27), (20, 25, 50),
                                   (96, 12, 10), (128, 16, 8)])
def test_x_transform_roundtrip(kw, shape):
    A, Simulation = kw
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=1, heterogeneous=False, nonlinear=False,
                         absorbing=False, pml=0)
    _banner("x roundtrip %s" % (shape,))
    sim = Simulation(scen)
    rng = np.random.default_rng(0)
    p = rng.standard_normal(nx * ny * nz).astype(np.float32)
    sim.set_field(A.KW_FIELD_P, p)
    back = sim.get_field(A.KW_FIELD_P)
    assert rel_l2(back, p) < 2e-6


@pytest.mark.parametrize("shape", [(48, 20, 18), (64, 64, 64), (40, 45, 27), (20, 25, 50),
                                   (32, 30, 24)])
def test_one_step_gradient_and_divergence(kw, shape):
    """One step from a random pressure: u = -dt/rho0 dp/dxi exercises the 3D
    r2c, the fused z gradient operator and the c2r; the new pressure adds the
    divergence chain.  Compared with the oracle's operators at 1e-5."""
    A, Simulation = kw
    nx, ny, nz = shape
    g = sc.Grid(nx, ny, nz, 1e-4, 1.1e-4, 0.9e-4, cfl=0.3, pml_size=(0, 0, 0))
    m = sc.Medium(1500.0, 1000.0, 0.0, 5.0, 1.5, nonlinear=False, absorbing=False)
    scen = sc.Scenario("grad_%dx%dx%d" % shape, g, m, None, sc.Sensor(record=0), 1)
    _banner(scen.name)
    sim = Simulation(scen)
    orc = Oracle(scen)
    rng = np.random.default_rng(3)
    p = rng.standard_normal(orc.shape).astype(np.float32)
    orc.set_pressure(p.astype(np.float64))
    sim.set_field(A.KW_FIELD_P, p)
    for f in (A.KW_FIELD_RHOX, A.KW_FIELD_RHOY, A.KW_FIELD_RHOZ):
        sim.set_field(f, (orc.rho[0]).astype(np.float32))
    orc.rho = [r.astype(np.float32).astype(np.float64) for r in orc.rho]
    sim.step(1)
    orc.step(1)
    for a, f in enumerate((A.KW_FIELD_UX, A.KW_FIELD_UY, A.KW_FIELD_UZ)):
        e = rel_l2(sim.get_field(f), orc.u[a])
        print("  u%d rel %.2e" % (a, e))
        assert e < 1e-5
    e = rel_l2(sim.get_field(A.KW_FIELD_P), orc.p)
    print("  p rel %.2e" % e)
    assert e < 1e-5


# ---------------------------------------------------------------------------
# full-step parity on seeded scenarios
# ---------------------------------------------------------------------------

SMALL = [
    dict(shape=(48, 20, 18), het=True, nl=True, ab=True, steps=30, mask=False),
    dict(shape=(64, 36, 30), het=True, nl=True, ab=True, steps=25, mask=True, ne=3),
    dict(shape=(40, 45, 27), het=True, nl=False, ab=False, steps=30, mask=False),
    dict(shape=(32, 32, 32), het=False, nl=False, ab=False, steps=40, mask=True),
    dict(shape=(20, 25, 50), het=True, nl=True, ab=False, steps=30, mask=False),
    dict(shape=(50, 16, 12), het=False, nl=False, ab=True, steps=30, mask=True),
    dict(shape=(96, 24, 20), het=True, nl=True, ab=True, steps=20, mask=False),
]


@pytest.mark.parametrize("case", SMALL, ids=["%dx%dx%d" % c["shape"] + ("_nl" if c["nl"] else "")
                                               + ("_ab" if c["ab"] else "") for c in SMALL])
def test_parity_small(kw, case):
    nx, ny, nz = case["shape"]
    scen = sc.small_case(nx, ny, nz, seed=7, heterogeneous=case["het"], nonlinear=case["nl"],
                         absorbing=case["ab"], pml=4, steps=case["steps"],
                         sensor_mask=case["mask"], n_elements=case.get("ne", 1))
    sim, orc = _run_both(kw, scen, case["steps"])
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


def test_parity_water_plane_64(kw):
    """64^3 water, 1 MHz plane source, 10-point PML, CFL 0.3, 200 steps."""
    scen = sc.water_plane(seed=0)
    sim, orc = _run_both(kw, scen, scen.steps)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


def test_graph_replay_matches_eager(kw):
    A, Simulation = kw
    scen = sc.small_case(48, 20, 18, seed=3, steps=24, sensor_mask=True)
    _banner("graph vs eager")
    s1 = Simulation(scen, graph_steps=0)
    s2 = Simulation(scen, graph_steps=8)
    s1.step(24)
    s2.step(24)
    for what in (A.KW_REC_P_FINAL, A.KW_REC_P_MAX, A.KW_REC_P_SERIES):
        a = s1.gather(what, device=False)
        b = s2.gather(what, device=False)
        assert np.array_equal(a, b), what


# ---------------------------------------------------------------------------
# exact solutions on the GPU (lossless homogeneous, no PML)
# ---------------------------------------------------------------------------

def _lossless(nx, ny, nz, cfl=0.3):
    g = sc.Grid(nx, ny, nz, 1e-4, 1e-4, 1e-4, cfl=cfl, pml_size=(0, 0, 0))
    m = sc.Medium(1500.0, 1000.0, 0.0, 5.0, 1.5, nonlinear=False, absorbing=False)
    return sc.Scenario("lossless_%dx%dx%d" % (nx, ny, nz), g, m, None,
                       sc.Sensor(record=sc.REC_P_FINAL | sc.REC_U_FINAL), 0)


def test_green_function_exact_gpu(kw):
    A, Simulation = kw
    nx, ny, nz = 32, 24, 20
    scen = _lossless(nx, ny, nz)
    _banner("green function %s" % scen.name)
    orc = Oracle(scen)       # used only for its wavenumber grid and dt
    rng = np.random.default_rng(5)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p0 = np.exp(-((x - 14.3) ** 2 + (y - 11.0) ** 2 + (z - 9.5) ** 2) / 6.0) * 1e5
    p0 += 1e3 * rng.standard_normal(p0.shape)
    p0 = p0.astype(np.float32).astype(np.float64)
    orc.set_pressure(p0)
    g = orc.pressure_gradient(p0)
    u0 = [orc.dt / (2 * 1000.0) * ga for ga in g]
    sim = Simulation(scen)
    sim.set_field(A.KW_FIELD_P, p0.astype(np.float32))
    for f, r in zip((A.KW_FIELD_RHOX, A.KW_FIELD_RHOY, A.KW_FIELD_RHOZ), orc.rho):
        sim.set_field(f, r.astype(np.float32))
    for f, u in zip((A.KW_FIELD_UX, A.KW_FIELD_UY, A.KW_FIELD_UZ), u0):
        sim.set_field(f, u.astype(np.float32))
    steps = 300
    sim.step(steps)
    expect = np.fft.ifftn(np.cos(1500.0 * orc.k * steps * orc.dt) * np.fft.fftn(p0)).real
    e = rel_l2(sim.get_field(A.KW_FIELD_P), expect)
    print("  green rel %.2e" % e)
    assert e < 1e-4


def test_plane_wave_exact_gpu(kw):
    A, Simulation = kw
    nx, ny, nz = 48, 40, 30
    scen = _lossless(nx, ny, nz)
    _banner("plane wave %s" % scen.name)
    orc = Oracle(scen)
    z, y, x = np.meshgrid(np.arange(nz) * 1e-4, np.arange(ny) * 1e-4, np.arange(nx) * 1e-4,
                          indexing="ij")
    kv = 2 * np.pi * np.array([3, 2, 1]) / (np.array([nx, ny, nz]) * 1e-4)
    k = np.linalg.norm(kv)
    A0, c0, rho0 = 2.0e5, 1500.0, 1000.0
    th = c0 * k * orc.dt
    p0 = A0 * np.cos(kv[0] * x + kv[1] * y + kv[2] * z)
    sim = Simulation(scen)
    sim.set_field(A.KW_FIELD_P, p0.astype(np.float32))
    for f in (A.KW_FIELD_RHOX, A.KW_FIELD_RHOY, A.KW_FIELD_RHOZ):
        sim.set_field(f, (p0 / (3 * c0 * c0)).astype(np.float32))
    for a, f in enumerate((A.KW_FIELD_UX, A.KW_FIELD_UY, A.KW_FIELD_UZ)):
        xs = [x, y, z]
        xs[a] = xs[a] + 0.5e-4
        u = A0 * kv[a] / (rho0 * c0 * k) * np.cos(kv[0] * xs[0] + kv[1] * xs[1] + kv[2] * xs[2]
                                                  + th / 2)
        sim.set_field(f, u.astype(np.float32))
    n = 400
    sim.step(n)
    expect = A0 * np.cos(kv[0] * x + kv[1] * y + kv[2] * z - n * th)
    e = rel_l2(sim.get_field(A.KW_FIELD_P), expect)
    print("  plane wave rel %.2e" % e)
    assert e < 1e-4


# ---------------------------------------------------------------------------
# failure detection
# ---------------------------------------------------------------------------

def test_nonfinite_pressure_is_reported(kw):
    A, Simulation = kw
    scen = sc.small_case(32, 16, 12, seed=2, steps=4)
    _banner("non-finite flag")
    sim = Simulation(scen)
    rho = np.zeros(scen.grid.npts, np.float32)
    rho[1234] = np.nan
    sim.set_field(A.KW_FIELD_RHOX, rho)
    sim.step(3)
    with pytest.raises(A.KwError) as ei:
        sim.gather(A.KW_REC_P_MAX, device=False)
    assert ei.value.code == A.KW_ENONFINITE
    assert sim.stats()["nonfinite_step"] == 1


def test_stats_counts(kw):
    A, Simulation = kw
    scen = sc.small_case(32, 16, 12, seed=2, steps=2)
    sim = Simulation(scen)
    sim.step(2)
    st = sim.stats()
    assert (st["fft_forward_per_step"], st["fft_inverse_per_step"]) == (6, 8)
    scen2 = sc.small_case(32, 16, 12, seed=2, steps=2, nonlinear=False, absorbing=False)
    st2 = Simulation(scen2).stats()
    assert st2["fft_forward_per_step"] + st2["fft_inverse_per_step"] == 10


# ---------------------------------------------------------------------------
# the 256^3 tissue workload at full size (few steps; oracle at 256^3 is slow)
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_parity_tissue_bowl_256_full_size(kw):
    scen = sc.tissue_bowl(seed=0, n=256, steps=3)
    scen.sensor.record |= sc.REC_P_FINAL | sc.REC_U_FINAL
    sim, orc = _run_both(kw, scen, 3, graph_steps=0)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


def test_fft_engines_and_schedules_agree(kw):
    """The same run with the fixed-width engine (default power-of-two plans),
    other fixed schedules, and the generic engine (radix-32 schedules) must
    agree to float32 round-off."""
    A, Simulation = kw
    scen = sc.small_case(64, 32, 64, seed=4, steps=12, sensor_mask=True)
    _banner("engines agree")
    ref = Simulation(scen)
    ref.step(12)
    p_ref = ref.gather(A.KW_REC_P_FINAL, device=False)
    for plans in ([(0, [8, 4]), (1, [8, 4]), (2, [8, 8])],
                  [(0, [32]), (1, [32]), (2, [32, 2])],
                  [(0, [2, 16]), (1, [4, 8]), (2, [4, 16])],
                  [(0, [4, 4, 2]), (1, [4, 4, 2]), (2, [4, 4, 4])]):
        sim = Simulation(scen)
        for axis, rad in plans:
            sim.set_plan(axis, rad)
        sim.step(12)
        e = rel_l2(sim.gather(A.KW_REC_P_FINAL, device=False), p_ref)
        print("  plans %s rel %.2e" % (plans, e))
        assert e < 1e-5


FOUR = [((32, 16, 64), [(0, [4, 4]), (1, [4, 4]), (2, [4, 4, 4])]),
        ((256, 12, 10), [(0, [4, 4, 4, 2])]),
        ((64, 20, 30), [(0, [4, 2, 4])])]


@pytest.mark.parametrize("shape,plans", FOUR, ids=["%dx%dx%d" % f[0] for f in FOUR])
def test_parity_four_wide_engine(kw, shape, plans):
    """The four-wide fixed engine (radices up to 4, 32 threads a 128-point
    row) on every pass kind, heterogeneous nonlinear absorbing medium with a
    mass source and a PML, against the oracle."""
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=5, heterogeneous=True, nonlinear=True, absorbing=True,
                         pml=3, steps=8, sensor_mask=False)
    sim, orc = _run_both(kw, scen, 8, plans=plans)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


# 1024-point y and z columns run in 1024-thread blocks of 16 columns; (40, 6,
# 1024) and (40, 1024, 6) have a full and a ragged tile of 16 columns
LONG = [(16, 8, 1024), (16, 1024, 8), (1024, 8, 8), (16, 8, 512), (32, 512, 6), (512, 6, 10),
        (16, 8, 256), (24, 10, 960), (40, 6, 1024), (40, 1024, 6)]


@pytest.mark.parametrize("shape", LONG, ids=["%dx%dx%d" % s for s in LONG])
def test_parity_long_axes(kw, shape):
    """Transforms of 256-1024 points (up to 64 threads per transform and three
    radix passes), with a heterogeneous nonlinear absorbing medium and a PML."""
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=9, heterogeneous=True, nonlinear=True, absorbing=True,
                         pml=2, steps=6, sensor_mask=False)
    sim, orc = _run_both(kw, scen, 6)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


# Plans whose passes all have one radix run on kernels built for that radix
# alone (16·16 for 256 points and 8·8·8 for 512 by default): the 16-wide on
# y columns and x rows, the 8-wide on y and z columns (z columns of 256 and x
# rows of 512 points are in the long-axis cases above); plans of radices 8
# and 4 (6 and 4) on the 8-wide (12-wide) kernels built for those two
SINGLE = [((16, 256, 8), []),
          ((512, 6, 8), [(0, [16, 16])]),
          ((16, 64, 512), [(1, [8, 8]), (2, [8, 8, 8])]),
          # radices 8 and 4 at width 8 (the 256^3 rows' schedule 8·4·4)
          ((256, 8, 6), [(0, [8, 4, 4])]),
          ((8, 128, 32), [(1, [8, 4, 4]), (2, [8, 4])]),
          # the 1024-thread blocks of these kernels (16 columns of 64 and of
          # 128 threads)
          ((16, 512, 8), [(1, [8, 8, 8])]),
          ((16, 8, 1024), [(2, [8, 8, 4, 4])]),
          # radices 6 and 4 at width 12 (the 192^3 rows' schedule)
          ((192, 12, 10), [(0, [6, 4, 4])]),
          ((40, 96, 24), [(1, [6, 4, 4]), (2, [6, 4])])]


@pytest.mark.parametrize("shape,plans", SINGLE, ids=["%dx%dx%d" % c[0] for c in SINGLE])
def test_parity_single_radix_engines(kw, shape, plans):
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=17, heterogeneous=True, nonlinear=True, absorbing=True,
                         pml=2, steps=6, sensor_mask=True)
    sim, orc = _run_both(kw, scen, 6, plans=plans)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


# Homogeneous absorbing water (scalar c0^2 tau, c0^2 eta): the merged
# absorption z pass (one inverse transform for both terms of Eq. (8)), which
# the 1024^3 water workload runs at 1024 points in half-width tiles, and the
# pressure kernel reading the merged spectrum with the mask-sensor code
# (kw_xeos<..., SENS, MERGED>, fixed x engine for nx >= 32)
MERGED = [(32, 8, 1024), (48, 6, 1024), (32, 1024, 6), (1024, 8, 8), (64, 36, 30)]


@pytest.mark.parametrize("shape", MERGED, ids=["%dx%dx%d" % s for s in MERGED])
def test_parity_merged_absorption(kw, shape):
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=13, heterogeneous=False, nonlinear=True,
                         absorbing=True, pml=2, steps=8, sensor_mask=True, amp=2e6)
    scen = scen.replace(name="merged_" + scen.name)
    sim, orc = _run_both(kw, scen, 8)
    st = sim.stats()
    assert st["fft_inverse_per_step"] == 7            # the merged path ran
    assert st["fft_forward_per_step"] == 5            # constant rho0: no transform of rho0 sum du
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


# Absorbing media with a constant rho0 and maps of c0 and alpha0: the
# divergence z pass forms the tau term's spectrum from the sum of the three
# divergence spectra (DIVA) and the absorption pass transforms rho alone
# (ABSR, terms kept apart since c0^2 tau and c0^2 eta are maps).  Fixed and
# generic z engines, even ny (double rows 0 and ny/2) and odd ny, 1024-point
# columns.
RHO0C = [(48, 20, 18), (64, 36, 30), (40, 45, 27), (32, 8, 1024), (32, 32, 32)]


@pytest.mark.parametrize("shape", RHO0C, ids=["%dx%dx%d" % s for s in RHO0C])
def test_parity_constant_rho0_absorbing(kw, shape):
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=17, heterogeneous=True, nonlinear=True,
                         absorbing=True, pml=2, steps=10, sensor_mask=True, amp=2e6)
    med = scen.medium
    scen = scen.replace(name="rho0c_" + scen.name,
                        medium=sc.Medium(med.c0, 1000.0, med.alpha0, med.bona, alpha_power=1.5,
                                         nonlinear=True, absorbing=True))
    sim, orc = _run_both(kw, scen, 10)
    st = sim.stats()
    assert (st["fft_forward_per_step"], st["fft_inverse_per_step"]) == (5, 8)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


# Lengths 2^a 3 and 2^a 5 on the mixed-radix fixed engine (12 or 20 elements
# per thread, radices dividing 12 or 20, butterfly groups of non-power-of-two
# size): x rows of 24, 40 and 48 points (density pass in three thread groups),
# y and z columns of 24 to 100 points, next to generic-engine axes; and the
# 32-wide fixed engine (radix-32 passes only) on x rows, y and z columns
# (1024 points in two passes), next to radix-32 schedules with a radix-2 pass,
# which run on the generic engine.
MIXED = [((48, 40, 36), [(0, [12, 2]), (1, [20, 2]), (2, [12, 3])]),
         # the 32-wide fixed engine (two radix-32 passes for 1024 points)
         ((16, 64, 1024), [(1, [32, 2]), (2, [32, 32])]),
         ((128, 32, 48), [(0, [32, 2]), (1, [32])]),
         ((64, 32, 48), [(0, [32]), (1, [32])]),
         ((80, 24, 60), [(0, [20, 2]), (1, [12, 2])]),
         ((96, 36, 40), [(0, [12, 4]), (1, [6, 6]), (2, [10, 4])]),
         ((40, 48, 100), [(1, [4, 4, 3]), (2, [20, 5])])]


@pytest.mark.parametrize("shape,plans", MIXED, ids=["%dx%dx%d" % c[0] for c in MIXED])
def test_parity_mixed_radix_engine(kw, shape, plans):
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=21, heterogeneous=True, nonlinear=True, absorbing=True,
                         pml=3, steps=12, sensor_mask=True, amp=2e6)
    scen = scen.replace(name="mixed_" + scen.name)
    sim, orc = _run_both(kw, scen, 12, plans=plans)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


@pytest.mark.slow
def test_water_bowl_1024_full_size_properties(kw):
    """The 1024^3 homogeneous water grid with the 3 MHz bowl, in the launch
    configuration bench.py times: the pressure stays finite and bounded, and
    it keeps the x <-> y exchange symmetry of the set-up (axis-centred bowl,
    isotropic spacing; the symmetry the scheme preserves exactly, pinned on the
    oracle) to float32 round-off.  The oracle itself cannot run at this size."""
    A, Simulation = kw
    scen = sc.water_bowl_large(n=1024, steps=40)
    _banner("water bowl 1024^3, 40 steps")
    sim = Simulation(scen)
    sim.step(40)
    st = sim.stats()
    assert st["nonfinite_step"] == -1
    p = sim.get_field(A.KW_FIELD_P).reshape(1024, 1024, 1024)
    pmax = float(np.abs(p).max())
    print("  max|p| %.3e" % pmax)
    assert 1e5 < pmax < 2e7
    # symmetry on a band of z-planes through the source (keeps host memory small)
    band = p[100:260]
    err = float(np.abs(band - band.transpose(0, 2, 1)).max() / np.abs(band).max())
    print("  x<->y symmetry error %.2e" % err)
    assert err < 1e-4


# ---------------------------------------------------------------------------
# checkpoint / restart (state snapshots)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mask,on_device", [(True, True), (False, False)])
def test_snapshot_resume_is_bitwise(kw, mask, on_device):
    """Run 30 steps straight, or 13 steps, snapshot, restore into a fresh
    simulation and run 17 more: every recorded output is bit-for-bit equal."""
    A, Simulation = kw
    scen = sc.small_case(40, 18, 24, seed=21, steps=30, sensor_mask=mask)
    _banner("snapshot resume mask=%s device=%s" % (mask, on_device))
    ref = Simulation(scen)
    ref.step(30)
    first = Simulation(scen)
    first.step(13)
    snap = first.save(device=on_device)
    first.close()
    second = Simulation(scen)
    second.load(snap)
    second.step(17)
    assert second.stats()["steps"] == 30
    whats = [A.KW_REC_P_FINAL, A.KW_REC_U_FINAL]
    whats += [A.KW_REC_P_SERIES] if mask else [A.KW_REC_P_MAX, A.KW_REC_P_RMS]
    for what in whats:
        a = ref.gather(what, device=False)
        b = second.gather(what, device=False)
        assert np.array_equal(a, b), what


def test_snapshot_rejects_other_setup(kw):
    A, Simulation = kw
    s1 = Simulation(sc.small_case(40, 18, 24, seed=21, steps=4))
    s1.step(2)
    snap = s1.save(device=False)
    s2 = Simulation(sc.small_case(40, 18, 20, seed=21, steps=4))
    with pytest.raises(A.KwError) as e:
        s2.load(snap)
    assert e.value.code == A.KW_EINVAL
    s3 = Simulation(sc.small_case(40, 18, 24, seed=21, steps=4))
    with pytest.raises(A.KwError) as e:
        s3.load(snap[: len(snap) // 2])
    assert e.value.code == A.KW_EINVAL
    bad = snap.copy()
    bad[:8] = 0
    with pytest.raises(A.KwError):
        s3.load(bad)


# ---------------------------------------------------------------------------
# on-device reductions: peak negative pressure, harmonic amplitudes, velocity
# series at mask points
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mask", [True, False])
def test_parity_pmin_harmonics_useries(kw, mask):
    A, Simulation = kw
    steps = 40
    scen = sc.small_case(48, 20, 18, seed=17, steps=steps, sensor_mask=mask, amp=2e6)
    rec = sc.REC_P_MIN | sc.REC_HARMONICS | sc.REC_P_MAX
    if mask:
        rec |= sc.REC_U_SERIES | sc.REC_P_SERIES
    scen = scen.replace(sensor=sc.Sensor(record=rec, index=scen.sensor.index if mask else None,
                                         record_start=9, series_capacity=steps, n_harmonics=3))
    scen = scen.replace(name=scen.name + ("_mask" if mask else "_all"))
    sim, orc = _run_both(kw, scen, steps)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    assert set(errs) >= {"p_min", "harmonics"}
    for k, e in errs.items():
        assert e <= tol, (k, e)
    # a snapshot round trip keeps the new accumulators too
    snap = sim.save(device=True)
    sim2 = Simulation(scen)
    sim2.load(snap)
    for what in (A.KW_REC_P_MIN, A.KW_REC_HARMONICS):
        assert np.array_equal(sim.gather(what, device=False), sim2.gather(what, device=False))


# ---------------------------------------------------------------------------
# source kinds: force on one velocity component, imposed pressure
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,axis,absorbing", [(1, 0, True), (1, 1, False), (1, 2, True),
                                                 (2, 0, True), (2, 0, False)])
def test_parity_source_kinds(kw, kind, axis, absorbing):
    A, Simulation = kw
    steps = 16
    scen = sc.small_case(40, 18, 20, seed=23, steps=steps, sensor_mask=True, amp=1e3,
                         absorbing=absorbing, n_elements=3)
    src = scen.source
    scale = 2e6 if kind == sc.SOURCE_PRESSURE else 1e6     # Pa, or m/s^2 (dt F ~ 0.02 m/s)
    scen = scen.replace(source=sc.Source(index=src.index, element=src.element,
                                         amp=(src.amp / 1e3 * scale).astype(np.float32),
                                         phase=src.phase, freq=src.freq, kind=kind, axis=axis),
                        name="kind%d_axis%d_%s" % (kind, axis, "abs" if absorbing else "lossless"))
    sim, orc = _run_both(kw, scen, steps)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


# ---------------------------------------------------------------------------
# edge cases: smallest and odd grids, the widest x row, degenerate set-ups
# ---------------------------------------------------------------------------

EDGE = [(4, 4, 4), (6, 5, 4), (8, 9, 5), (10, 15, 25), (2048, 4, 4), (4, 6, 2 * 3 * 5 * 5)]


@pytest.mark.parametrize("shape", EDGE, ids=["%dx%dx%d" % s for s in EDGE])
def test_parity_edge_shapes(kw, shape):
    """Minimum sizes (two-point x spectra), odd y and z lengths (no Nyquist row
    or plane), the longest x row (1024-point x transforms) and a mixed-radix z."""
    nx, ny, nz = shape
    scen = sc.small_case(nx, ny, nz, seed=31, heterogeneous=True, nonlinear=True,
                         absorbing=True, pml=1, steps=8, sensor_mask=False)
    sim, orc = _run_both(kw, scen, 8)
    errs, tol = compare_outputs(sim, orc, scen, REPORT)
    for k, e in errs.items():
        assert e <= tol, (k, e)


def test_degenerate_setups(kw):
    A, Simulation = kw
    base = sc.small_case(24, 10, 12, seed=3, steps=6)
    _banner("degenerate set-ups")
    # zero drive: every field stays exactly zero
    src = base.source
    zero = base.replace(source=sc.Source(index=src.index, amp=np.zeros(1, np.float32),
                                         phase=src.phase, freq=src.freq))
    sim = Simulation(zero)
    sim.step(6)
    assert not np.any(sim.gather(A.KW_REC_P_FINAL, device=False))
    assert not np.any(sim.gather(A.KW_REC_U_FINAL, device=False))
    # no source and no sensor: steps run, the final fields are readable
    sim = Simulation(base.replace(source=None, sensor=sc.Sensor(record=0)))
    sim.step(3)
    assert not np.any(sim.get_field(A.KW_FIELD_P))
    # zero steps, then recorded quantities of an empty window
    sim = Simulation(base.replace(sensor=sc.Sensor(record=sc.REC_P_RMS | sc.REC_P_MAX,
                                                   record_start=100)))
    sim.step(0)
    sim.step(4)
    assert not np.any(sim.gather(A.KW_REC_P_RMS, device=False))
    assert np.all(np.isneginf(sim.gather(A.KW_REC_P_MAX, device=False)))
