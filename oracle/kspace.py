"""FP64 CPU oracle of the k-space pseudospectral time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module: it exists so that the tests, the smoke check and the CPU
baseline of the benchmark can compare the HIP library against a plain, slow,
obviously correct implementation written straight from the paper
(Jaros, Rendell & Treeby, "Full-wave nonlinear ultrasound simulation on
distributed clusters with applications in high-intensity focused
ultrasound", Section 2.2, Eqs. (4a)-(4d), (5), (6), (8)).

Everything is float64.  3D arrays have numpy shape (nz, ny, nx) (x fastest).
The FFTs are full complex transforms over all three axes (no half-spectrum
tricks): FT is the unnormalised forward DFT and IFT includes 1/N, as in numpy.

Where the paper does not fix a detail, the oracle takes these readings (each
is also listed in the design notes):
  * sinc is the unnormalised sin(x)/x, with sinc(0) = 1 (kappa, Section 2.2).
  * c_ref defaults to max(c0); dt defaults to cfl * min(spacing) / max(c0).
  * PML (Berenger split field, not specified further in the paper): inside the
    grid, n points per side, sigma(d) = alpha * (c_ref / spacing) * (d / n)^4
    with d the depth into the layer in grid points (staggered points at
    half-integer depths); factor P = exp(-sigma dt / 2) applied twice:
        u   <- P+ (P+ u - dt / rho0+ dp)
        rho <- P  (P rho - dt rho0 du) / (1 + 2 dt du)       (+ dt M)
  * rho0 on the staggered grid along an axis is the mean of the two
    neighbours; the last point along that axis keeps its own value.
  * The pressure drive s (Pa) enters as an additive mass source split evenly
    over the three density components, M_xi = 2 s / (3 c0 dx), added after the
    division of Eq. (4d), sampled at t = (n + 1/2) dt:
        s_e(n+1/2) = a_e sin(2 pi f (n + 1/2) dt + phi_e).
  * Other source kinds: a force per unit mass F on one velocity component
    (the F term of Eq. (4b)), u += dt F after the update, sampled at t = n dt;
    a pressure source imposes p^(n+1) = s at its points after the equation of
    state, sampled at t = (n + 1) dt, leaving the densities as they are.
  * k^(y-2) and k^(y-1) are set to 0 at k = 0.
  * Absorption coefficient: alpha0 [Np (rad/s)^-y m^-1]
        = 100 alpha0[dB/(MHz^y cm)] / (20 log10 e) / (2 pi 1e6)^y.
  * Sensors record p^(n+1) after every step whose number n+1 >= record_start.

Parity unpinned (no closed form or invariant fixes these readings; they are
checked only as GPU = oracle): the PML profile constants, the interpolation
of rho0 to the staggered points, the bowl voxelisation and the source time
sampling.
"""
from __future__ import annotations

import os
from typing import Optional

import numpy as np
import scipy.fft as sfft

_WORKERS = os.cpu_count() or 1


def wavenumbers(n: int, spacing: float) -> np.ndarray:
    """Eq. (5): the set of wavenumbers along one axis, returned in FFT order
    (zero frequency first) so that it lines up with the DFT output."""
    if n % 2 == 0:
        m = np.arange(-n // 2, n // 2)
    else:
        m = np.arange(-(n - 1) // 2, (n - 1) // 2 + 1)
    k = m * (2.0 * np.pi / (spacing * n))
    return np.fft.ifftshift(k)


def alpha_db_to_neper(alpha_db, y: float):
    """dB / (MHz^y cm)  ->  Np (rad/s)^-y m^-1 (units stated with Eq. (3))."""
    return 100.0 * np.asarray(alpha_db, np.float64) / (20.0 * np.log10(np.e)) \
        / (2.0 * np.pi * 1.0e6) ** y


def pml_profile(n: int, size: int, alpha: float, c_ref: float, spacing: float,
                dt: float, staggered: bool) -> np.ndarray:
    """1D split-field PML factor exp(-sigma dt/2) along one axis."""
    if size <= 0 or alpha == 0.0:
        return np.ones(n)
    i = np.arange(n, dtype=np.float64) + (0.5 if staggered else 0.0)
    depth_left = size - i
    depth_right = i - (n - 1 - size)
    d = np.maximum(np.maximum(depth_left, depth_right), 0.0)
    sigma = alpha * (c_ref / spacing) * (d / size) ** 4
    return np.exp(-sigma * dt / 2.0)


def staggered_mean(a: np.ndarray, axis: int) -> np.ndarray:
    """Value midway between neighbours along `axis`; the last point keeps its
    own value."""
    a = np.asarray(a, np.float64)
    out = a.copy()
    lo = [slice(None)] * 3
    hi = [slice(None)] * 3
    lo[axis] = slice(0, -1)
    hi[axis] = slice(1, None)
    out[tuple(lo)] = 0.5 * (a[tuple(lo)] + a[tuple(hi)])
    return out


def _field(v, shape) -> np.ndarray:
    if np.isscalar(v) or np.ndim(v) == 0:
        return np.full(shape, float(v), np.float64)
    a = np.asarray(v, np.float64)
    assert a.shape == shape, (a.shape, shape)
    return a


class Oracle:
    """One simulation.  Construct from a scenario (see the scenario module's
    data classes), then call step()."""

    def __init__(self, scen, workers: Optional[int] = None):
        self.workers = workers or _WORKERS
        g, m = scen.grid, scen.medium
        self.grid, self.medium = g, m
        shape = (g.nz, g.ny, g.nx)
        self.shape = shape
        self.N = g.nx * g.ny * g.nz
        self.spacing = (g.dx, g.dy, g.dz)          # xi = x, y, z
        self.axis = (2, 1, 0)                      # numpy axis of x, y, z

        self.c0 = _field(m.c0, shape)
        self.rho0 = _field(m.rho0, shape)
        self.bona = _field(m.bona, shape)
        self.nonlinear = bool(m.nonlinear)
        self.absorbing = bool(m.absorbing)
        cmax = float(self.c0.max())
        self.c_ref = float(m.c_ref) if m.c_ref > 0 else cmax
        self.dt = float(g.dt) if g.dt > 0 else g.cfl * min(g.dx, g.dy, g.dz) / cmax
        dt = self.dt

        # wavenumber grids, broadcast to (nz, ny, nx)
        kvec = [wavenumbers(g.nx, g.dx), wavenumbers(g.ny, g.dy), wavenumbers(g.nz, g.dz)]
        self.kvec = kvec
        kx = kvec[0][None, None, :]
        ky = kvec[1][None, :, None]
        kz = kvec[2][:, None, None]
        kb = (kx, ky, kz)
        k = np.sqrt(kx * kx + ky * ky + kz * kz)
        self.k = k
        # kappa = sinc(c_ref k dt / 2), unnormalised sinc
        self.kappa = np.sinc(self.c_ref * k * dt / 2.0 / np.pi)
        # Eq. (4a) and (4c): i k_xi exp(+- i k_xi dxi / 2)
        self.d_plus = [1j * kb[a] * np.exp(+1j * kb[a] * self.spacing[a] / 2.0) for a in range(3)]
        self.d_minus = [1j * kb[a] * np.exp(-1j * kb[a] * self.spacing[a] / 2.0) for a in range(3)]

        # Eq. (3) coefficients and Eq. (8) fractional Laplacians
        y = float(m.alpha_power)
        self.y = y
        if self.absorbing:
            a0 = alpha_db_to_neper(_field(m.alpha0, shape), y)
            self.tau = -2.0 * a0 * self.c0 ** (y - 1.0)
            self.eta = 2.0 * a0 * self.c0 ** y * np.tan(np.pi * y / 2.0)
            with np.errstate(divide="ignore"):
                self.k_tau = np.where(k > 0, k ** (y - 2.0), 0.0)
                self.k_eta = np.where(k > 0, k ** (y - 1.0), 0.0)

        # PML factors on the regular and staggered grid, per axis
        self.pml = []
        self.pml_stag = []
        n_ax = (g.nx, g.ny, g.nz)
        for a in range(3):
            shp = [1, 1, 1]
            shp[self.axis[a]] = n_ax[a]
            reg = pml_profile(n_ax[a], int(g.pml_size[a]), float(g.pml_alpha[a]), self.c_ref,
                              self.spacing[a], dt, staggered=False)
            stg = pml_profile(n_ax[a], int(g.pml_size[a]), float(g.pml_alpha[a]), self.c_ref,
                              self.spacing[a], dt, staggered=True)
            self.pml.append(reg.reshape(shp))
            self.pml_stag.append(stg.reshape(shp))

        # ambient density at the staggered points of each velocity component
        self.rho0_stag = [staggered_mean(self.rho0, self.axis[a]) for a in range(3)]

        # source
        src = scen.source
        self.src = None
        if src is not None and len(src.index) > 0:
            idx = np.asarray(src.index, np.int64)
            elem = (np.zeros(idx.size, np.int64) if src.element is None
                    else np.asarray(src.element, np.int64))
            c_at = self.c0.reshape(-1)[idx]
            self.src = dict(idx=idx, elem=elem,
                            coef=2.0 / (3.0 * c_at * g.dx),
                            amp=np.asarray(src.amp, np.float64),
                            phase=np.asarray(src.phase, np.float64),
                            freq=float(src.freq),
                            signal=None if src.signal is None
                            else np.asarray(src.signal, np.float64),
                            kind=int(getattr(src, "kind", 0)), axis=int(getattr(src, "axis", 0)))

        # optional tape for the discrete adjoint (oracle/adjoint.py): when a
        # list, every step appends the values its reverse pass needs
        self.tape = None

        # state: p^n, u^(n-1/2), rho_xi^n
        self.p = np.zeros(shape)
        self.u = [np.zeros(shape) for _ in range(3)]
        self.rho = [np.zeros(shape) for _ in range(3)]
        self.n = 0

        # sensors
        sen = scen.sensor
        self.sensor_index = None if sen.index is None else np.asarray(sen.index, np.int64)
        self.record_start = int(sen.record_start)
        nrec = self.N if self.sensor_index is None else self.sensor_index.size
        self.p_max = np.full(nrec, -np.inf)
        self.p_min = np.full(nrec, np.inf)
        self.p_sum2 = np.zeros(nrec)
        self.n_rec = 0
        self.series = []
        self.u_series = []
        # harmonic sums: sum over recorded m of p^m exp(-i h w m dt), h = 1..H
        self.n_harm = int(getattr(sen, "n_harmonics", 0) or 0)
        f = float(getattr(sen, "harmonic_freq", 0.0) or 0.0)
        if f <= 0.0 and scen.source is not None:
            f = float(scen.source.freq)
        self.harm_freq = f
        self.harm = np.zeros((self.n_harm, nrec), np.complex128)
        self.fft_forward = 0
        self.fft_inverse = 0

    # -- transforms (counted, so the per-step FFT count can be checked) -----
    def ft(self, a):
        self.fft_forward += 1
        return sfft.fftn(a, workers=self.workers)

    def ift(self, a):
        self.fft_inverse += 1
        return sfft.ifftn(a, workers=self.workers).real

    # -- initial conditions --------------------------------------------------
    def set_pressure(self, p0, split=None):
        """Set p^0.  The density components are set so that their sum obeys
        the linear equation of state, p0 / c0^2, split by `split` (default
        equal thirds)."""
        p0 = np.asarray(p0, np.float64).reshape(self.shape)
        split = (1.0 / 3, 1.0 / 3, 1.0 / 3) if split is None else split
        self.p = p0.copy()
        for a in range(3):
            self.rho[a] = split[a] * p0 / (self.c0 ** 2)

    def set_velocity(self, ux, uy, uz):
        """Set u^(-1/2) on the staggered grid."""
        self.u = [np.asarray(v, np.float64).reshape(self.shape).copy() for v in (ux, uy, uz)]

    # -- the time step ---------------------------------------------------------
    def source_values(self, n: int, offset: float = 0.5) -> np.ndarray:
        """Drive value of each element in step n, at t = (n + offset) dt (the
        sampled signal gives sample n whatever the offset)."""
        s = self.src
        if s["signal"] is not None:
            sig = s["signal"]
            return sig[:, n] if n < sig.shape[1] else np.zeros(sig.shape[0])
        t = (n + offset) * self.dt
        return s["amp"] * np.sin(2.0 * np.pi * s["freq"] * t + s["phase"])

    def pressure_gradient(self, p):
        """Eq. (4a): d p / d xi at the points shifted by +dxi/2, for xi = x, y, z.
        One forward transform is shared by the three components."""
        P = self.ft(p)
        return [self.ift(self.d_plus[a] * self.kappa * P) for a in range(3)]

    def velocity_divergence(self, u):
        """Eq. (4c): d u_xi / d xi back on the regular grid, per component."""
        return [self.ift(self.d_minus[a] * self.kappa * self.ft(u[a])) for a in range(3)]

    def step(self, nsteps: int = 1, progress=None):
        """Advance nsteps steps; progress(i), if given, is called after each."""
        for i in range(nsteps):
            self._one_step()
            if progress is not None:
                progress(i + 1)

    def _one_step(self):
        dt = self.dt
        # (4a) pressure gradient on the staggered grid
        grad = self.pressure_gradient(self.p)
        # (4b) velocity update, with the split-field PML
        for a in range(3):
            q = self.pml_stag[a]
            self.u[a] = q * (q * self.u[a] - dt / self.rho0_stag[a] * grad[a])
        # force source (the F term of Eq. (4b)), sampled at t = n dt
        if self.src is not None and self.src["kind"] == 1:
            s = self.src
            flat = self.u[s["axis"]].reshape(-1)
            np.add.at(flat, s["idx"], dt * self.source_values(self.n, 0.0)[s["elem"]])
        # (4c) velocity divergence, one component at a time
        div = self.velocity_divergence(self.u)
        # (4d) split density update (nonlinear denominator), PML, mass source
        for a in range(3):
            q = self.pml[a]
            num = q * (q * self.rho[a] - dt * self.rho0 * div[a])
            if self.nonlinear:
                num = num / (1.0 + 2.0 * dt * div[a])
            self.rho[a] = num
        if self.src is not None and self.src["kind"] == 0:
            s = self.src
            add = dt * s["coef"] * self.source_values(self.n)[s["elem"]]
            for a in range(3):
                flat = self.rho[a].reshape(-1)
                np.add.at(flat, s["idx"], add)
        rho = self.rho[0] + self.rho[1] + self.rho[2]
        if self.tape is not None:
            self.tape.append(dict(n=self.n, div=[d.copy() for d in div],
                                  rho_parts=[r.copy() for r in self.rho], rho=rho.copy()))
        # (8) absorption and dispersion through the fractional Laplacians
        if self.absorbing:
            dudt_term = self.ift(self.k_tau * self.ft(self.rho0 * (div[0] + div[1] + div[2])))
            disp_term = self.ift(self.k_eta * self.ft(rho))
            L_d = -self.tau * dudt_term + self.eta * disp_term
        else:
            L_d = 0.0
        # (6) equation of state
        if self.nonlinear:
            self.p = self.c0 ** 2 * (rho + self.bona / (2.0 * self.rho0) * rho * rho - L_d)
        else:
            self.p = self.c0 ** 2 * (rho - L_d)
        # pressure source: p^(n+1) imposed at the points, t = (n + 1) dt
        if self.src is not None and self.src["kind"] == 2:
            s = self.src
            self.p.reshape(-1)[s["idx"]] = self.source_values(self.n, 1.0)[s["elem"]]
        self.n += 1
        if self.tape is not None:
            self.tape[-1]["p"] = self.p.copy()
        self._record()

    def _record(self):
        if self.n < self.record_start:
            return
        flat = self.p.reshape(-1)
        v = flat if self.sensor_index is None else flat[self.sensor_index]
        self.p_max = np.maximum(self.p_max, v)
        self.p_min = np.minimum(self.p_min, v)
        self.p_sum2 += v * v
        self.n_rec += 1
        if self.sensor_index is not None:
            self.series.append(v.copy())
            # u^(n-1/2) is recorded together with p^n
            self.u_series.append(np.stack([u.reshape(-1)[self.sensor_index] for u in self.u]))
        t = self.n * self.dt
        for h in range(self.n_harm):
            self.harm[h] += v * np.exp(-1j * (h + 1) * 2.0 * np.pi * self.harm_freq * t)

    # -- outputs ---------------------------------------------------------------
    @property
    def p_rms(self) -> np.ndarray:
        return np.sqrt(self.p_sum2 / max(self.n_rec, 1))

    def p_series(self) -> np.ndarray:
        return np.array(self.series) if self.series else np.zeros((0, 0))

    def u_series_array(self) -> np.ndarray:
        """[recorded steps, 3, sensor points]."""
        return np.array(self.u_series) if self.u_series else np.zeros((0, 3, 0))

    def harmonics(self) -> np.ndarray:
        """Complex amplitudes A_h = (2/N) sum_m p^m exp(-i h w t_m), [H, points]."""
        return 2.0 * self.harm / max(self.n_rec, 1)

    def intensity(self) -> np.ndarray:
        """Time-mean of p^2 / (rho0 c0) over the recorded steps."""
        rc = (self.rho0 * self.c0).reshape(-1)
        if self.sensor_index is not None:
            rc = rc[self.sensor_index]
        return self.p_sum2 / max(self.n_rec, 1) / rc
