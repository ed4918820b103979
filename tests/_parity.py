"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import numpy as np

from paper_1408_4675_amd import scenarios as sc


def rel_l2(gpu, ref):
    gpu = np.asarray(gpu, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(gpu - ref) / den) if den > 0 else float(np.linalg.norm(gpu))


def tolerance(scen):
    """rel L2 budget per recorded field: 1e-4 linear lossless, 1e-3 nonlinear or absorbing."""
    return 1e-3 if (scen.medium.nonlinear or scen.medium.absorbing) else 1e-4


def compare_outputs(sim, orc, scen, report, tol=None):
    """Compare every recorded field of a GPU run with the oracle; return the
    dict of rel L2 errors (also appended to `report`)."""
    from paper_1408_4675_amd import _abi as A
    tol = tolerance(scen) if tol is None else tol
    errs = {}
    rec = scen.sensor.record
    if rec & sc.REC_P_FINAL:
        errs["p_final"] = rel_l2(sim.gather(A.KW_REC_P_FINAL, device=False), orc.p)
    if rec & sc.REC_U_FINAL:
        u = sim.gather(A.KW_REC_U_FINAL, device=False).reshape(3, -1)
        for a, nm in enumerate("xyz"):
            errs["u%s_final" % nm] = rel_l2(u[a], orc.u[a])
    if rec & sc.REC_P_MAX:
        errs["p_max"] = rel_l2(sim.gather(A.KW_REC_P_MAX, device=False), orc.p_max)
    if rec & sc.REC_P_RMS:
        errs["p_rms"] = rel_l2(sim.gather(A.KW_REC_P_RMS, device=False), orc.p_rms)
    if rec & sc.REC_P_SERIES:
        ser = sim.gather(A.KW_REC_P_SERIES, device=False)
        ref = orc.p_series()[: scen.sensor.series_capacity]
        errs["p_series"] = rel_l2(ser, ref)
    if rec & sc.REC_INTENSITY:
        errs["intensity"] = rel_l2(sim.gather(A.KW_REC_INTENSITY, device=False), orc.intensity())
    if rec & sc.REC_P_MIN:
        errs["p_min"] = rel_l2(sim.gather(A.KW_REC_P_MIN, device=False), orc.p_min)
    if rec & sc.REC_HARMONICS:
        h = sim.gather(A.KW_REC_HARMONICS, device=False).reshape(scen.sensor.n_harmonics, -1, 2)
        ref = orc.harmonics()
        errs["harmonics"] = rel_l2(np.stack([h[..., 0], h[..., 1]]),
                                   np.stack([ref.real, ref.imag]))
    if rec & sc.REC_U_SERIES:
        u = sim.gather(A.KW_REC_U_SERIES, device=False)
        ref = orc.u_series_array()[: scen.sensor.series_capacity]
        errs["u_series"] = rel_l2(u, ref)
    report.append((scen.name, errs, tol))
    print("parity %-28s tol %.0e  %s" % (scen.name, tol,
          "  ".join("%s %.2e" % kv for kv in errs.items())), flush=True)
    return errs, tol
