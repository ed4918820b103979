"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch each one.  A pin set that every mutant passes would prove nothing."""
import numpy as np
import pytest

import oracle.kspace as ok
from tests import test_oracle_pins as pins


def _mutant(mutate):
    real = ok.Oracle

    def factory(*a, **k):
        o = real(*a, **k)
        mutate(o)
        return o
    return factory


def _normalised_sinc(o):
    o.kappa = np.sinc(o.c_ref * o.k * o.dt / 2.0)


def _swap_shift_signs(o):
    o.d_plus, o.d_minus = o.d_minus, o.d_plus


def _no_kappa(o):
    o.kappa = np.ones_like(o.kappa)


def _unstaggered_density(o):
    o.rho0_stag = [o.rho0.copy() for _ in range(3)]


def _full_bona(o):                 # B/A where B/(2A) belongs
    o.bona = 2.0 * o.bona


def _tau_sign(o):
    if o.absorbing:
        o.tau = -o.tau


def _swap_fractional_powers(o):
    if o.absorbing:
        o.k_tau, o.k_eta = o.k_eta, o.k_tau


def _eta_dropped(o):
    if o.absorbing:
        o.eta = 0.0 * o.eta


def _source_scale(o):
    if o.src is not None:
        o.src["coef"] = 0.5 * o.src["coef"]


def _transposed_axes(o):           # x and y wavenumbers exchanged on a non-cubic grid
    o.d_plus = [o.d_plus[1], o.d_plus[0], o.d_plus[2]]


def _override(**members):
    """Mutant that replaces methods or properties of the class of `o`."""
    def mutate(o):
        o.__class__ = type("Mutant", (type(o),), members)
    return mutate


def _rms_no_sqrt_fn(self):
    return self.p_sum2 / max(self.n_rec, 1)


def _rms_extra_count_fn(self):
    return np.sqrt(self.p_sum2 / (self.n_rec + 1))


def _intensity_c0_squared_fn(self):
    rc = (self.rho0 * self.c0 ** 2).reshape(-1)
    if self.sensor_index is not None:
        rc = rc[self.sensor_index]
    return self.p_sum2 / max(self.n_rec, 1) / rc


def _record_one_step_early(self):
    # the window opens one step before record_start
    self.record_start -= 1
    ok.Oracle._record(self)
    self.record_start += 1


def _record_peak_magnitude(self):
    # |p| where the peak positive pressure belongs
    before = self.p_max.copy()
    ok.Oracle._record(self)
    if self.n >= self.record_start:
        flat = self.p.reshape(-1)
        v = flat if self.sensor_index is None else flat[self.sensor_index]
        self.p_max = np.maximum(before, np.abs(v))


_rms_no_sqrt = _override(p_rms=property(_rms_no_sqrt_fn))
_rms_no_sqrt.__name__ = "_rms_no_sqrt"
_rms_extra_count = _override(p_rms=property(_rms_extra_count_fn))
_rms_extra_count.__name__ = "_rms_extra_count"
_intensity_c0_squared = _override(intensity=_intensity_c0_squared_fn)
_intensity_c0_squared.__name__ = "_intensity_c0_squared"
_window_early = _override(_record=_record_one_step_early)
_window_early.__name__ = "_window_early"
_peak_magnitude = _override(_record=_record_peak_magnitude)
_peak_magnitude.__name__ = "_peak_magnitude"


MUTANTS = [
    (_normalised_sinc, [lambda: pins.test_green_function_exact((12, 10, 16), 400)]),
    (_no_kappa, [lambda: pins.test_oblique_plane_wave_exact()]),
    (_swap_shift_signs, [lambda: pins.test_oblique_plane_wave_exact()]),
    (_unstaggered_density, [lambda: pins.test_energy_conserved_heterogeneous_lossless()]),
    (_full_bona, [lambda: pins.test_fubini_harmonics_pre_shock()]),
    (_tau_sign, [lambda: pins.test_single_mode_follows_two_by_two_recurrence(1.5, 20.0)]),
    (_swap_fractional_powers, [lambda: pins.test_single_mode_follows_two_by_two_recurrence(1.5, 20.0)]),
    (_eta_dropped, [lambda: pins.test_absorption_rate_and_dispersion_match_power_law(1.5)]),
    (_source_scale, [lambda: pins.test_plane_source_emits_its_drive_amplitude()]),
    (_transposed_axes, [lambda: pins.test_gradient_is_exact_shifted_derivative((1, 2, 3))]),
    (_rms_no_sqrt, [lambda: pins.test_aggregates_of_exact_plane_wave(False)]),
    (_rms_extra_count, [lambda: pins.test_aggregates_of_exact_plane_wave(False)]),
    (_intensity_c0_squared, [lambda: pins.test_aggregates_of_exact_plane_wave(True)]),
    (_window_early, [lambda: pins.test_aggregates_follow_exact_green_function_series()]),
    (_peak_magnitude, [lambda: pins.test_aggregates_follow_exact_green_function_series()]),
]


@pytest.mark.parametrize("mutate,checks", MUTANTS, ids=[m[0].__name__ for m in MUTANTS])
def test_pins_catch_mutant(monkeypatch, mutate, checks):
    monkeypatch.setattr(pins, "Oracle", _mutant(mutate))
    caught = False
    for chk in checks:
        try:
            with np.errstate(all="ignore"):
                chk()
        except (AssertionError, FloatingPointError, ValueError):
            caught = True
    assert caught, "mutant %s survived its pins" % mutate.__name__
