"""Oracle parity of the full-size workloads, written as committed records.

    python tests/full_size_parity.py c1 --out profiles/parity_water_plane_64.json
    python tests/full_size_parity.py c2 --steps 100 --out profiles/parity_tissue_bowl_256.json
    python tests/full_size_parity.py c3 --n 512 --steps 10 --out profiles/parity_water_bowl_512.json
    python tests/full_size_parity.py c5 --out profiles/parity_adjoint_bowl_128.json

c1: 64^3 water, plane source, 200 steps; c2: 256^3 layered tissue with the
bowl; c3: the 1024^3 water workload scaled to n^3 (same spacing, bowl and
time step; 1024^3 itself is beyond the host's memory for the FP64 oracle);
c5: the focusing-objective gradient on the 128^3 tissue bowl with 64
elements and 600 steps against the FP64 discrete adjoint.  The GPU runs in
the launch configuration the benchmark times (captured graphs, autotuned
plans); every recorded field is compared with the FP64 oracle by relative L2
(1e-4 linear lossless, 1e-3 nonlinear or absorbing), and the record states
each error.  Needs a GPU and, for c2/c3/c5, tens of GB of host memory.
Test infrastructure: it runs the oracle."""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import Oracle                                    # noqa: E402
from paper_1408_4675_amd import scenarios as sc              # noqa: E402
from tests._parity import compare_outputs, rel_l2, tolerance  # noqa: E402


def log(msg):
    print("[parity] " + msg, flush=True)


def host():
    mem = None
    with open("/proc/meminfo") as fh:
        for line in fh:
            if line.startswith("MemTotal:"):
                mem = round(int(line.split()[1]) / 2 ** 20, 1)
    return dict(nproc=os.cpu_count(), ram_gib=mem)


def every(k, what, t0):
    def cb(i):
        if i % k == 0:
            log("%s: %d done, %.0f s" % (what, i, time.perf_counter() - t0))
    return cb


def forward_record(scen, steps):
    from paper_1408_4675_amd.simulation import Simulation
    log("%s: GPU, %d steps" % (scen.name, steps))
    t0 = time.perf_counter()
    sim = Simulation(scen)
    sim.step(steps)
    sim.synchronize()
    gpu_s = time.perf_counter() - t0
    log("%s: oracle" % scen.name)
    t0 = time.perf_counter()
    orc = Oracle(scen)
    orc.step(steps, every(max(1, steps // 20), "oracle steps", t0))
    cpu_s = time.perf_counter() - t0
    report = []
    errs, tol = compare_outputs(sim, orc, scen, report)
    plans = dict(sim.plans)
    sim.close()
    return dict(workload=scen.name, grid=[scen.grid.nx, scen.grid.ny, scen.grid.nz],
                steps=steps, nonlinear=scen.medium.nonlinear, absorbing=scen.medium.absorbing,
                heterogeneous=not np.isscalar(scen.medium.c0),
                launch="captured graphs of 8 steps, autotuned plans %s" % plans,
                rel_l2=errs, tolerance=tol, passed=all(e <= tol for e in errs.values()),
                gpu_s=round(gpu_s, 2), oracle_s=round(cpu_s, 1))


def adjoint_record():
    from oracle.adjoint import AdjointOracle
    from paper_1408_4675_amd.adjoint import focus_gradient, with_drive
    scen, focus = sc.adjoint_bowl(seed=0)
    w = sc.focal_weights(scen.grid, focus, 2e-3)
    rng = np.random.default_rng(1)
    ne = len(scen.source.amp)
    scen = with_drive(scen, rng.uniform(0.5e6, 1.5e6, ne), rng.uniform(-np.pi, np.pi, ne))
    log("adjoint: GPU gradient (checkpoints every 50 steps)")
    t0 = time.perf_counter()
    out = focus_gradient(scen, w, checkpoint_every=50)
    gpu_s = time.perf_counter() - t0
    log("adjoint: FP64 oracle forward")
    t0 = time.perf_counter()
    ref = AdjointOracle(scen, w)
    Jr = ref.forward(every(50, "oracle forward steps", t0))
    log("adjoint: FP64 oracle reverse")
    gr = ref.backward(every(50, "oracle reverse steps", t0))
    cpu_s = time.perf_counter() - t0
    errs = dict(J=abs(out["J"] - Jr) / abs(Jr), dJ_damp=rel_l2(out["grad_amp"], gr["grad_amp"]),
                dJ_dphase=rel_l2(out["grad_phase"], gr["grad_phase"]),
                dJ_ds=rel_l2(out["source_gradient"], gr["dJds"]))
    log("adjoint: " + "  ".join("%s %.2e" % kv for kv in errs.items()))
    return dict(workload="adjoint_bowl_128: 128^3 tissue (seed 0), 64-element bowl, 600 steps, "
                         "intensity over the last 200 steps, 2 mm focal sphere",
                elements=ne, steps=scen.steps, checkpoint_every=50, J_gpu=out["J"], J_fp64=Jr,
                rel_l2=errs, tolerance=1e-3, passed=all(e <= 1e-3 for e in errs.values()),
                gpu_s=round(gpu_s, 2), oracle_s=round(cpu_s, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.case == "c1":
        scen = sc.water_plane(seed=0)
        rec = forward_record(scen, a.steps or scen.steps)
    elif a.case == "c2":
        steps = a.steps or 100
        scen = sc.tissue_bowl(seed=0, n=256, steps=steps)
        scen.sensor.record |= sc.REC_P_FINAL | sc.REC_U_FINAL
        rec = forward_record(scen, steps)
    elif a.case == "c3":
        # the 1024^3 water set-up at n^3 (same spacing, bowl scaled, same dt);
        # within the few steps the oracle affords the wave moves a fraction of
        # a millimetre, so the recorded series is taken on a block of points
        # around the bowl apex that the wave crosses (at the focus, 15 mm away
        # at n = 512, the series would hold only round-off)
        steps = a.steps or 20
        scen = sc.water_bowl_large(n=a.n, steps=steps)
        g = scen.grid
        apex = int(round(3e-3 * a.n / 512 / g.dz))
        c = a.n // 2
        ix, iy, iz = np.meshgrid(np.arange(c - 2, c + 3), np.arange(c - 2, c + 3),
                                 np.arange(apex - 4, apex + 13), indexing="ij")
        idx = np.unique(sc.flat_index(g, ix.ravel(), iy.ravel(), iz.ravel()).astype(np.int64))
        scen = scen.replace(sensor=sc.Sensor(record=sc.REC_P_SERIES | sc.REC_P_MAX | sc.REC_P_FINAL
                                             | sc.REC_U_FINAL, index=idx,
                                             series_capacity=steps))
        rec = forward_record(scen, steps)
        rec["sensor"] = "%d points around the bowl apex (axis x = y = %d, z = %d..%d)" % (
            idx.size, c, apex - 4, apex + 12)
    else:
        rec = adjoint_record()
    rec["host"] = host()
    rec["command"] = "python " + " ".join(sys.argv)
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    log("wrote %s: passed=%s" % (a.out, rec["passed"]))
    return 0 if rec["passed"] else 1


if __name__ == "__main__":
    sys.exit(main())
