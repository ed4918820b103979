"""The FP64 discrete adjoint of the oracle, pinned by central finite
differences of the FP64 forward model (the objective of the focusing
problem: mean intensity in a sphere minus the mean outside)."""
import numpy as np
import pytest

from oracle.adjoint import AdjointOracle, objective
from paper_1408_4675_amd import scenarios as sc


def _case(nonlinear, absorbing, heterogeneous, pml=3, steps=30, seed=4, n=(18, 16, 20)):
    scen = sc.small_case(*n, seed=seed, heterogeneous=heterogeneous, nonlinear=nonlinear,
                         absorbing=absorbing, pml=pml, steps=steps, amp=2.0e6, n_elements=4)
    scen = scen.replace(sensor=sc.Sensor(record=sc.REC_INTENSITY, record_start=steps - 12))
    w = sc.focal_weights(scen.grid, (n[0] // 2, n[1] // 2, n[2] // 2), 3.5e-4)
    return scen, w


def _with(scen, amp=None, phase=None):
    src = scen.source
    return scen.replace(source=sc.Source(index=src.index, element=src.element,
                                         amp=src.amp if amp is None else amp.astype(np.float32),
                                         phase=src.phase if phase is None
                                         else phase.astype(np.float32), freq=src.freq))


@pytest.mark.parametrize("nonlinear,absorbing,heterogeneous",
                         [(False, False, False), (True, False, True), (True, True, True)])
def test_adjoint_matches_central_differences(nonlinear, absorbing, heterogeneous):
    scen, w = _case(nonlinear, absorbing, heterogeneous)
    adj = AdjointOracle(scen, w, workers=4)
    adj.forward()
    g = adj.backward()
    amp = scen.source.amp.astype(np.float64)
    ph = scen.source.phase.astype(np.float64)
    for e in range(len(amp)):
        h = 1e-3 * amp[e]
        # float32 source arrays: step on values exactly representable around amp
        ap, am = amp.copy(), amp.copy()
        ap[e] += h
        am[e] -= h
        ap32, am32 = ap.astype(np.float32), am.astype(np.float32)
        fd = (objective(_with(scen, amp=ap32), w, 4) - objective(_with(scen, amp=am32), w, 4)) \
            / (float(ap32[e]) - float(am32[e]))
        assert abs(fd - g["grad_amp"][e]) <= 1e-6 * abs(fd) + 1e-12 * abs(adj.J), (e, fd, g["grad_amp"][e])
        hp = 1e-3
        pp, pm = ph.copy(), ph.copy()
        pp[e] += hp
        pm[e] -= hp
        pp32, pm32 = pp.astype(np.float32), pm.astype(np.float32)
        fdp = (objective(_with(scen, phase=pp32), w, 4) - objective(_with(scen, phase=pm32), w, 4)) \
            / (float(pp32[e]) - float(pm32[e]))
        assert abs(fdp - g["grad_phase"][e]) <= 2e-5 * abs(fdp) + 1e-9 * abs(adj.J), \
            (e, fdp, g["grad_phase"][e])


def test_adjoint_of_quadratic_objective_is_exact_in_the_linear_case():
    """Linear lossless medium: J is a quadratic form in the amplitudes, so
    J(2a) = 4 J(a) and the Euler identity sum_e a_e dJ/da_e = 2 J holds exactly."""
    scen, w = _case(False, False, True)
    adj = AdjointOracle(scen, w, workers=4)
    J = adj.forward()
    g = adj.backward()
    amp = scen.source.amp.astype(np.float64)
    assert abs(float(np.dot(amp, g["grad_amp"])) - 2.0 * J) <= 1e-10 * abs(J)
    J2 = objective(_with(scen, amp=2 * scen.source.amp), w, 4)
    assert abs(J2 - 4 * J) <= 1e-10 * abs(J)


# planted mistakes in the reverse pass (source-level edits of a private copy of
# the module): the finite-difference pin must catch each one
MUTANTS = [
    ("+ 2.0 * dt * (t[\"rho_parts\"][a] - add)", ""),                     # drop the d/d(den) term
    ("db_common = o.rho0 * self._op(o.k_tau, ab)", "db_common = 0.0 * ab"),  # drop the tau path
    ("rb_tot = rb_tot + self._op(o.k_eta, bb)", "rb_tot = rb_tot"),          # drop the eta path
    ("rb[a] = R * q * q / den", "rb[a] = R * q / den"),                      # one PML factor
    ("(1.0 + o.bona / o.rho0 * rho)", "(1.0 + 0.5 * o.bona / o.rho0 * rho)"),  # B/2A for B/A
    ("np.conj(o.d_minus[a] * o.kappa)", "o.d_minus[a] * o.kappa"),          # no transpose
    ("gb.append(-q * dt", "gb.append(q * dt"),                               # sign of Eq. (4b)
]


@pytest.mark.parametrize("old,new", MUTANTS)
def test_adjoint_mutants_are_caught(old, new, tmp_path):
    import importlib.util
    import os
    import oracle.adjoint as ref
    src = open(ref.__file__).read()
    assert old in src
    path = os.path.join(str(tmp_path), "adjoint_mutant.py")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new).replace("from .kspace import Oracle",
                                               "from oracle.kspace import Oracle"))
    spec = importlib.util.spec_from_file_location("adjoint_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    scen, w = _case(True, True, True, steps=24)
    good = AdjointOracle(scen, w, workers=4)
    good.forward()
    g_ref = good.backward()
    bad = mod.AdjointOracle(scen, w, workers=4)
    bad.forward()
    g_bad = bad.backward()
    # the reference agrees with finite differences to ~1e-6 (test above); a
    # mutant must be visibly off on some parameter
    diff = max(np.max(np.abs(g_bad["grad_amp"] - g_ref["grad_amp"]) / np.max(np.abs(g_ref["grad_amp"]))),
               np.max(np.abs(g_bad["grad_phase"] - g_ref["grad_phase"]) / np.max(np.abs(g_ref["grad_phase"]))))
    assert diff > 1e-5, diff
