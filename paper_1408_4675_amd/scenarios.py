"""Seeded synthetic inputs for the k-space pseudospectral solver.

This module builds *data only*: grids, medium property maps, source and
sensor index lists.  It contains none of the solver's arithmetic (no
wavenumbers, no k-space operators, no unit conversion of the absorption
coefficient, no time-step rule); both the HIP library and the CPU oracle
consume what it produces and each implements the method on its own.

Array convention: 3D arrays have numpy shape (nz, ny, nx) in C order, so the
flat index of grid point (x, y, z) is x + nx*(y + ny*z) (x fastest).  Medium
maps are float32 because the library takes float32 host arrays; the oracle
widens the same values to float64.

The paper's media come from a patient CT set (Section 5) and its benchmark
media are only described as fully heterogeneous (Section 4.1).  The layered
tissue generator below is a seeded stand-in with the sound-speed, density,
absorption and nonlinearity ranges of soft tissue; water surrounds the
transducer as in the paper's application (Section 5).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple, Union

import numpy as np

Scalar = float
MapOrScalar = Union[float, np.ndarray]

# recorded-quantity bits; the same values are defined in include/kw.h
REC_P_MAX = 1
REC_P_RMS = 2
REC_P_SERIES = 4
REC_P_FINAL = 8
REC_U_FINAL = 16
REC_INTENSITY = 32
REC_P_MIN = 64
REC_HARMONICS = 128
REC_U_SERIES = 256

# source kinds; the same values are defined in include/kw.h
SOURCE_MASS = 0
SOURCE_FORCE = 1
SOURCE_PRESSURE = 2

# water, the coupling medium of the paper's application (Section 5)
WATER = dict(c0=1500.0, rho0=1000.0, alpha0=0.75, bona=5.0)


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float = 0.0            # 0 -> derived from cfl by the solver
    cfl: float = 0.3
    pml_size: Tuple[int, int, int] = (10, 10, 10)
    pml_alpha: Tuple[float, float, float] = (2.0, 2.0, 2.0)

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Medium:
    c0: MapOrScalar            # sound speed [m/s]
    rho0: MapOrScalar          # ambient density [kg/m^3]
    alpha0: MapOrScalar        # absorption prefactor [dB / (MHz^y cm)]
    bona: MapOrScalar          # nonlinearity parameter B/A
    alpha_power: float = 1.5   # power-law exponent y
    c_ref: float = 0.0         # 0 -> max(c0)
    nonlinear: bool = True
    absorbing: bool = True


@dataclass
class Source:
    """Drive at the listed grid points: a pressure injected as a mass source
    (the default), a force per unit mass on one velocity component, or a
    pressure imposed on the points (kind)."""
    index: np.ndarray                      # int64, sorted, unique flat indices
    amp: np.ndarray                        # float32 per element [Pa]
    phase: np.ndarray                      # float32 per element [rad]
    freq: float = 1.0e6                    # [Hz]
    element: Optional[np.ndarray] = None   # int32 per point (None -> element 0)
    signal: Optional[np.ndarray] = None    # float32 [n_elements, n_samples]
    kind: int = 0                          # SOURCE_MASS, SOURCE_FORCE or SOURCE_PRESSURE
    axis: int = 0                          # velocity component of a force source

    @property
    def n_elements(self) -> int:
        return int(len(self.amp))


@dataclass
class Sensor:
    record: int = REC_P_MAX | REC_P_RMS
    index: Optional[np.ndarray] = None     # None -> every grid point
    record_start: int = 1                  # first step number whose pressure is recorded
    series_capacity: int = 0
    n_harmonics: int = 0                   # harmonics 1..n of harmonic_freq (REC_HARMONICS)
    harmonic_freq: float = 0.0             # 0 -> the source frequency


@dataclass
class Scenario:
    name: str
    grid: Grid
    medium: Medium
    source: Optional[Source]
    sensor: Sensor
    steps: int

    def replace(self, **kw) -> "Scenario":
        return dataclasses.replace(self, **kw)


def empty_source() -> Source:
    return Source(index=np.zeros(0, np.int64), amp=np.zeros(1, np.float32),
                  phase=np.zeros(1, np.float32), freq=1.0e6)


# ---------------------------------------------------------------------------
# geometry helpers (pure index bookkeeping)
# ---------------------------------------------------------------------------

def flat_index(grid: Grid, ix, iy, iz) -> np.ndarray:
    return (np.asarray(ix, np.int64) + grid.nx * (np.asarray(iy, np.int64)
            + grid.ny * np.asarray(iz, np.int64)))


def plane_source_z(grid: Grid, iz: int) -> np.ndarray:
    """Every (x, y) point of the plane z = iz, sorted."""
    iy, ix = np.meshgrid(np.arange(grid.ny), np.arange(grid.nx), indexing="ij")
    return np.sort(flat_index(grid, ix.ravel(), iy.ravel(), np.full(ix.size, iz)))


def bowl_points(grid: Grid, apex_z: float, radius: float, aperture: float,
                centre_xy: Optional[Tuple[float, float]] = None,
                n_rings: int = 1, n_sectors: int = 1) -> Tuple[np.ndarray, np.ndarray]:
    """Voxelise a spherical cap (focused bowl) whose axis is +z.

    A grid point g belongs to the bowl when its distance to the focus f
    differs from the radius by at most half a grid spacing, its distance from
    the axis is at most the aperture radius, and it lies on the transducer side
    of the focus.  The paper only says a 3D midpoint-circle style
    voxelisation was used (Section 5); this rule is a documented stand-in.

    Elements: n_rings equal-area rings (bands of r_perp^2) times n_sectors
    azimuthal sectors.  Returns (sorted flat indices, element id per point).
    """
    h = grid.dx
    if centre_xy is None:
        centre_xy = ((grid.nx // 2) * grid.dx, (grid.ny // 2) * grid.dy)
    fx, fy, fz = centre_xy[0], centre_xy[1], apex_z + radius
    a = 0.5 * aperture
    cap_h = radius - np.sqrt(max(radius * radius - a * a, 0.0))
    z_lo = int(np.floor((apex_z - h) / grid.dz))
    z_hi = int(np.ceil((apex_z + cap_h + h) / grid.dz))
    z_lo, z_hi = max(z_lo, 0), min(z_hi, grid.nz - 1)
    iz = np.arange(z_lo, z_hi + 1)
    iy = np.arange(grid.ny)
    ix = np.arange(grid.nx)
    Z, Y, X = np.meshgrid(iz * grid.dz, iy * grid.dy, ix * grid.dx, indexing="ij")
    rx, ry, rz = X - fx, Y - fy, Z - fz
    dist = np.sqrt(rx * rx + ry * ry + rz * rz)
    rperp2 = rx * rx + ry * ry
    on = (np.abs(dist - radius) <= 0.5 * h) & (rperp2 <= a * a) & (rz < 0)
    kk, jj, ii = np.nonzero(on)
    idx = flat_index(grid, ii, jj, iz[kk])
    ring = np.minimum((rperp2[on] / (a * a) * n_rings).astype(np.int64), n_rings - 1)
    ang = np.mod(np.arctan2(ry[on], rx[on]), 2 * np.pi)
    sector = np.minimum((ang / (2 * np.pi) * n_sectors).astype(np.int64), n_sectors - 1)
    on_axis = rperp2[on] == 0.0
    sector[on_axis] = 0
    elem = (ring * n_sectors + sector).astype(np.int32)
    order = np.argsort(idx, kind="stable")
    return idx[order], elem[order]


# ---------------------------------------------------------------------------
# media
# ---------------------------------------------------------------------------

TISSUE_RANGES = dict(c0=(1450.0, 1650.0), rho0=(950.0, 1100.0),
                     alpha0=(0.5, 1.5), bona=(5.0, 9.0))


def layered_tissue(grid: Grid, rng: np.random.Generator, water_until_z: float,
                   ranges=TISSUE_RANGES) -> dict:
    """Water up to water_until_z, then 3-6 tissue layers along z with smooth,
    sinusoidally perturbed interfaces, plus 2-6 Gaussian inclusions.
    Returns float32 maps of shape (nz, ny, nx) for c0, rho0, alpha0, bona."""
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    Lx, Ly, Lz = nx * grid.dx, ny * grid.dy, nz * grid.dz
    x = np.arange(nx) * grid.dx
    y = np.arange(ny) * grid.dy
    z = np.arange(nz) * grid.dz
    n_layers = int(rng.integers(3, 7))
    # interface mean depths: the first at the end of the water standoff
    inner = np.sort(rng.uniform(water_until_z + 0.1 * (Lz - water_until_z), Lz,
                                n_layers - 1))
    zbar = np.concatenate([[water_until_z], inner])
    names = ("c0", "rho0", "alpha0", "bona")
    vals = {n: [WATER[n]] + list(rng.uniform(ranges[n][0], ranges[n][1], n_layers))
            for n in names}
    X, Y = np.meshgrid(x, y, indexing="xy")      # (ny, nx)
    width = 2.0 * grid.dz
    out = {n: np.full((nz, ny, nx), vals[n][0], np.float64) for n in names}
    for j, zb in enumerate(zbar):
        surf = np.full((ny, nx), zb)
        if j > 0:
            for _ in range(3):
                A = rng.uniform(0.0, 1.0e-3) / 3.0
                kx, ky = 0, 0
                while kx == 0 and ky == 0:
                    kx, ky = int(rng.integers(0, 4)), int(rng.integers(0, 4))
                phi = rng.uniform(0, 2 * np.pi)
                surf = surf + A * np.sin(2 * np.pi * (kx * X / Lx + ky * Y / Ly) + phi)
        step = 0.5 * (1.0 + np.tanh((z[:, None, None] - surf[None]) / width))
        for n in names:
            out[n] += (vals[n][j + 1] - vals[n][j]) * step
    n_inc = int(rng.integers(2, 7))
    Z3 = z[:, None, None]
    for _ in range(n_inc):
        cx, cy = rng.uniform(0.2 * Lx, 0.8 * Lx), rng.uniform(0.2 * Ly, 0.8 * Ly)
        cz = rng.uniform(zbar[0] + 0.1 * (Lz - zbar[0]), Lz)
        sg = rng.uniform(1.0e-3, 3.0e-3)
        r2 = ((x[None, None, :] - cx) ** 2 + (y[None, :, None] - cy) ** 2 + (Z3 - cz) ** 2)
        g = np.exp(-r2 / (2 * sg * sg)) * (Z3 > water_until_z)
        for n in names:
            lo, hi = ranges[n]
            out[n] += rng.uniform(-0.5, 0.5) * (hi - lo) * g
    for n in names:
        lo, hi = ranges[n]
        tissue = Z3 + 0 * out[n] > water_until_z
        out[n] = np.where(tissue, np.clip(out[n], min(lo, WATER[n]), max(hi, WATER[n])), out[n])
        out[n] = out[n].astype(np.float32)
    return out


def random_medium(grid: Grid, rng: np.random.Generator, smooth: int = 2) -> dict:
    """Smooth random heterogeneous maps within the tissue ranges (for tests)."""
    out = {}
    for n, (lo, hi) in TISSUE_RANGES.items():
        f = rng.standard_normal(grid.shape)
        for ax in range(3):
            for _ in range(smooth):
                f = 0.25 * np.roll(f, 1, ax) + 0.5 * f + 0.25 * np.roll(f, -1, ax)
        f = (f - f.min()) / max(f.max() - f.min(), 1e-30)
        out[n] = (lo + (hi - lo) * f).astype(np.float32)
    return out


# ---------------------------------------------------------------------------
# the five workload configurations
# ---------------------------------------------------------------------------

def water_plane(seed: int = 0, n: int = 64, steps: int = 200) -> Scenario:
    """64^3 water, 0.1 mm spacing, 1 MHz plane source on z = 12 with a seeded
    amplitude in 0.5-2 MPa, 10-point PML, CFL 0.3, 200 steps."""
    rng = np.random.default_rng(seed)
    g = Grid(n, n, n, 1e-4, 1e-4, 1e-4, dt=0.0, cfl=0.3, pml_size=(10, 10, 10))
    med = Medium(**WATER, alpha_power=1.5)
    amp = np.array([rng.uniform(0.5e6, 2.0e6)], np.float32)
    src = Source(index=plane_source_z(g, 12), amp=amp, phase=np.zeros(1, np.float32),
                 freq=1.0e6)
    sen = Sensor(record=REC_P_MAX | REC_P_RMS | REC_P_FINAL | REC_U_FINAL)
    return Scenario("water_plane_%d" % n, g, med, src, sen, steps)


def tissue_bowl(seed: int = 0, n: int = 256, steps: int = 1000, dx: float = 1e-4,
                amp: float = 5.0e6, pml: int = 20) -> Scenario:
    """n^3 layered tissue with a 1 MHz focused bowl.  At n = 256 the bowl has a
    15 mm radius and 18 mm aperture with its apex 3 mm into the grid; at other
    n the geometry scales by n/256."""
    rng = np.random.default_rng(seed)
    g = Grid(n, n, n, dx, dx, dx, dt=0.0, cfl=0.3, pml_size=(pml, pml, pml))
    s = n / 256.0 * (dx / 1e-4)
    R, ap, apex = 15e-3 * s, 18e-3 * s, 3e-3 * s
    cap_h = R - np.sqrt(R * R - (ap / 2) ** 2)
    maps = layered_tissue(g, rng, water_until_z=apex + cap_h + 1e-3 * s)
    med = Medium(maps["c0"], maps["rho0"], maps["alpha0"], maps["bona"], alpha_power=1.5)
    idx, _ = bowl_points(g, apex, R, ap)
    src = Source(index=idx, amp=np.array([amp], np.float32), phase=np.zeros(1, np.float32),
                 freq=1.0e6)
    sen = Sensor(record=REC_P_MAX | REC_P_RMS)
    return Scenario("tissue_bowl_%d" % n, g, med, src, sen, steps)


def water_bowl_large(n: int = 1024, dx: float = 5e-5, steps: int = 100) -> Scenario:
    """n^3 homogeneous water at 0.05 mm, 3 MHz 2 MPa bowl (R 30 mm, aperture
    36 mm, apex 6 mm at n = 1024), 20-point PML, one focal sensor point."""
    g = Grid(n, n, n, dx, dx, dx, dt=1.0e-8, cfl=0.0, pml_size=(20, 20, 20))
    s = n / 1024.0
    R, ap, apex = 30e-3 * s, 36e-3 * s, 6e-3 * s
    med = Medium(**WATER, alpha_power=1.5)
    idx, _ = bowl_points(g, apex, R, ap)
    src = Source(index=idx, amp=np.array([2.0e6], np.float32),
                 phase=np.zeros(1, np.float32), freq=3.0e6)
    fz = int(round((apex + R) / g.dz))
    focus = flat_index(g, [n // 2], [n // 2], [min(fz, n - 1)])
    sen = Sensor(record=REC_P_SERIES, index=focus.astype(np.int64), series_capacity=steps)
    return Scenario("water_bowl_%d" % n, g, med, src, sen, steps)


def adjoint_bowl(seed: int = 0, n: int = 128, steps: int = 600,
                 n_rings: int = 8, n_sectors: int = 8) -> Tuple[Scenario, np.ndarray]:
    """128^3 seeded tissue, 64-element bowl (R 8 mm, aperture 10 mm, apex
    1.5 mm).  Returns the scenario and the focus grid position (ix, iy, iz)."""
    rng = np.random.default_rng(seed)
    g = Grid(n, n, n, 1e-4, 1e-4, 1e-4, dt=0.0, cfl=0.3, pml_size=(10, 10, 10))
    R, ap, apex = 8e-3, 10e-3, 1.5e-3
    cap_h = R - np.sqrt(R * R - (ap / 2) ** 2)
    maps = layered_tissue(g, rng, water_until_z=apex + cap_h + 1e-3)
    med = Medium(maps["c0"], maps["rho0"], maps["alpha0"], maps["bona"], alpha_power=1.5)
    idx, elem = bowl_points(g, apex, R, ap, n_rings=n_rings, n_sectors=n_sectors)
    ne = n_rings * n_sectors
    src = Source(index=idx, element=elem, amp=np.full(ne, 1.0e6, np.float32),
                 phase=np.zeros(ne, np.float32), freq=1.0e6)
    sen = Sensor(record=REC_INTENSITY, record_start=steps - 200 + 1)
    focus = np.array([n // 2, n // 2, int(round((apex + R) / g.dz))])
    return Scenario("adjoint_bowl_%d" % n, g, med, src, sen, steps), focus


def focal_weights(grid: Grid, focus: Sequence[int], radius: float) -> np.ndarray:
    """Weights w of the focusing objective sum_x w(x) I(x): +1/|S_in| at the
    points within `radius` [m] of the focus (grid indices ix, iy, iz), -1/|S_out|
    at every other point outside the PML, 0 in the PML.  Flat float64 array."""
    z, y, x = np.meshgrid(np.arange(grid.nz) * grid.dz, np.arange(grid.ny) * grid.dy,
                          np.arange(grid.nx) * grid.dx, indexing="ij")
    fx, fy, fz = focus[0] * grid.dx, focus[1] * grid.dy, focus[2] * grid.dz
    inside = (x - fx) ** 2 + (y - fy) ** 2 + (z - fz) ** 2 <= radius * radius
    core = np.zeros(grid.shape, bool)
    px, py, pz = grid.pml_size
    core[pz:grid.nz - pz, py:grid.ny - py, px:grid.nx - px] = True
    inside &= core
    outside = core & ~inside
    w = np.zeros(grid.shape)
    if inside.any():
        w[inside] = 1.0 / inside.sum()
    if outside.any():
        w[outside] = -1.0 / outside.sum()
    return w.reshape(-1)


SERVING_SIZES = (64, 96, 128, 160, 192, 256)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    scenario: Scenario


def serving_trace(seed: int = 0, n_requests: int = 200, rate: float = 20.0,
                  sizes: Sequence[int] = SERVING_SIZES, medium_pool: Optional[int] = None,
                  steps_range: Tuple[int, int] = (300, 1500)) -> List[Request]:
    """Poisson arrivals; per request a cubic grid from `sizes`, a seeded
    layered medium, a bowl scaled with the grid, 0.5-6 MPa and a step count
    drawn from `steps_range` (inclusive); p_max and p_rms recorded at every
    point.  With `medium_pool` = K, each size has K seeded media that requests
    of that size share (the draw of the request picks one), which bounds the
    host time and memory of building a long trace."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    pool: Dict[Tuple[int, int], Scenario] = {}
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(np.asarray(sizes)))
        amp = float(rng.uniform(0.5e6, 6.0e6))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        mseed = int(rng.integers(0, 2**31 - 1))
        pml = 10 if n < 128 else 20
        if medium_pool:
            key = (n, mseed % medium_pool)
            if key not in pool:
                pool[key] = tissue_bowl(seed=key[1], n=n, steps=1, pml=pml)
            base = pool[key]
            src = dataclasses.replace(base.source, amp=np.array([amp], np.float32))
            sc = base.replace(source=src, steps=steps)
        else:
            sc = tissue_bowl(seed=mseed, n=n, steps=steps, amp=amp, pml=pml)
        out.append(Request(rid, t, sc.replace(name="req%03d_%d" % (rid, n))))
    return out


def small_case(nx: int, ny: int, nz: int, seed: int = 0, heterogeneous: bool = True,
               nonlinear: bool = True, absorbing: bool = True, pml: int = 3,
               steps: int = 8, amp: float = 1.0e6, sensor_mask: bool = False,
               n_elements: int = 1) -> Scenario:
    """A small grid with a seeded random medium and a few random source
    points: the building block of the parity tests.  With sensor_mask the
    sensor is 17 random points with a pressure time series; otherwise every
    point is recorded (p_max, p_rms)."""
    rng = np.random.default_rng(seed)
    g = Grid(nx, ny, nz, 1e-4, 1.2e-4, 0.9e-4, dt=0.0, cfl=0.3, pml_size=(pml, pml, pml))
    if heterogeneous:
        maps = random_medium(g, rng)
        med = Medium(maps["c0"], maps["rho0"], maps["alpha0"], maps["bona"],
                     alpha_power=1.5, nonlinear=nonlinear, absorbing=absorbing)
    else:
        med = Medium(**WATER, alpha_power=1.5, nonlinear=nonlinear, absorbing=absorbing)
    npts = max(1, g.npts // 50)
    idx = np.unique(rng.integers(0, g.npts, npts).astype(np.int64))
    elem = rng.integers(0, n_elements, idx.size).astype(np.int32) if n_elements > 1 else None
    src = Source(index=idx, element=elem,
                 amp=rng.uniform(0.5, 1.0, n_elements).astype(np.float32) * amp,
                 phase=rng.uniform(-np.pi, np.pi, n_elements).astype(np.float32),
                 freq=1.0e6)
    if sensor_mask:
        sidx = np.unique(rng.integers(0, g.npts, 17).astype(np.int64))
        sen = Sensor(record=REC_P_MAX | REC_P_RMS | REC_P_SERIES | REC_P_FINAL | REC_U_FINAL,
                     index=sidx, record_start=1, series_capacity=steps)
    else:
        sen = Sensor(record=REC_P_MAX | REC_P_RMS | REC_P_FINAL | REC_U_FINAL,
                     index=None, record_start=1)
    return Scenario("small_%dx%dx%d" % (nx, ny, nz), g, med, src, sen, steps)
