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
