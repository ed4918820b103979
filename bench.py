"""Throughput of the k-space pseudospectral time step on one MI355X.

Workload (the headline configuration): 256^3 layered heterogeneous tissue,
nonlinear and absorbing, 1 MHz focused bowl at 5 MPa, 20-point PML, p_max and
p_rms recorded at every grid point, float32.  A second line item times the
1024^3 homogeneous water grid (3 MHz bowl, one focal sensor).

Prints one JSON line.  `value` = grid-point updates per second at 256^3 with
every input resident in HBM, timed over exactly `steps` steps run the
production way (captured HIP graphs).  A second region of the same length runs
with HIP events around every kernel on the simulation's stream; the roofline
of the dominant kernel class comes from it (algorithmic bytes per launch /
average duration).
The CPU baseline times the FP64 oracle on a bounded sample of the same 256^3
workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def measured_traffic(kernel_class, npts):
    """HBM bytes per launch of `kernel_class` from a committed rocprofv3 PMC
    summary (profiles/pmc_traffic*.json) taken on the current kernel sources
    and on a grid of `npts` points (the workload being reported); else None."""
    import glob
    from paper_1408_4675_amd.profiling import kernel_source_hash
    h = kernel_source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "pmc_traffic*.json"))):
        with open(path) as fh:
            d = json.load(fh)
        if d.get("source_hash") != h or d.get("points") != npts:
            continue
        k = d.get("kernels", {}).get(kernel_class)
        return None if k is None else k.get("hbm_bytes_per_launch")
    return None


def time_workload(scen, steps, warmup):
    """Warm up, time exactly `steps` steps the production way (captured HIP
    graphs, no instrumentation) for the throughput, then run `steps` more with
    HIP events around every kernel on the simulation's stream for the
    per-kernel durations.  Returns (graph seconds, profiled seconds, stats of
    the profiled region)."""
    import torch
    from paper_1408_4675_amd.simulation import Simulation
    sim = Simulation(scen)
    sim.step(warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.stats()                     # resolve anything pending
    sim.profile(True)
    base = sim.stats()["classes"]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    t3 = time.perf_counter()
    stats = sim.stats()
    sim.profile(False)
    for k, v in stats["classes"].items():
        v["ms"] -= base[k]["ms"]
        v["launches"] -= base[k]["launches"]
    # nonfinite check (also proves the run produced finite pressures)
    if stats["nonfinite_step"] >= 0:
        raise RuntimeError("non-finite pressure at step %d" % stats["nonfinite_step"])
    sim.close()
    return (t1 - t0), (t3 - t2), stats


def roofline(stats, npts):
    classes = {k: v for k, v in stats["classes"].items() if v["launches"] > 0}
    dom = max(classes, key=lambda k: classes[k]["ms"])
    c = classes[dom]
    avg_s = c["ms"] / c["launches"] / 1e3
    achieved = c["bytes"] / avg_s / 1e9
    per_class = {k: dict(ms_per_launch=round(v["ms"] / v["launches"], 5),
                         launches=v["launches"],
                         algorithmic_bytes=v["bytes"],
                         gbs=round(v["bytes"] / (v["ms"] / v["launches"] / 1e3) / 1e9, 1)
                         if v["bytes"] > 0 else None)
                 for k, v in classes.items()}
    return dom, dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                     frac=round(achieved / HBM_PEAK_GBS, 4),
                     traffic=measured_traffic(dom, npts),
                     kernel=dom, algorithmic_bytes_per_launch=c["bytes"],
                     avg_launch_ms=round(avg_s * 1e3, 5)), per_class


def pass_model_bytes(stats):
    """Algorithmic bytes of one step: sum over kernels of bytes x launches."""
    tot_b, steps = 0.0, None
    for k, v in stats["classes"].items():
        tot_b += v["bytes"] * v["launches"]
    return tot_b


def copy_ceiling(mib=1024, reps=10):
    """Device-to-device copy bandwidth (read + write bytes / time): the
    practical HBM ceiling the kernels are compared against."""
    import torch
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gbs = 2 * n * 4 * reps / dt / 1e9
    del a, b
    return round(gbs, 1)


def host_info():
    mem_gb = None
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), ram_gib=mem_gb)


# The paper's own CPU-cluster throughput, derived from its run times (context
# only: other hardware, other precision of the statement, I/O included).
PAPER_CONTEXT = [
    dict(what="largest benchmark, 4096x2048x2048 points, 25,000 steps projected at about 4.5 "
              "days on 1024 cores (Section 4.5)",
         grid_point_updates_per_s=1.1e9, cores=1024),
    dict(what="kidney application, 2048x1536x1536 points, 19,800 steps in 31 h 20 min on 768 "
              "cores including I/O and restarts (Section 5)",
         grid_point_updates_per_s=8.48e8, cores=768),
]


def cpu_scaling(sizes=(64, 128, 256), steps=3):
    """The FP64 oracle at several sizes, on all host cores and on one core
    (median step time after one warm-up step)."""
    from oracle import Oracle
    from paper_1408_4675_amd import scenarios as sc
    out = []
    for n in sizes:
        scen = sc.tissue_bowl(seed=0, n=n, steps=steps + 1)
        for workers in (os.cpu_count(), 1):
            o = Oracle(scen, workers=workers)
            o.step(1)
            ts = []
            for _ in range(steps):
                t0 = time.perf_counter()
                o.step(1)
                ts.append(time.perf_counter() - t0)
            med = float(np.median(ts))
            out.append(dict(n=n, cores=workers, s_per_step=round(med, 4),
                            grid_point_updates_per_s=round(scen.grid.npts / med, 1)))
            log("oracle %d^3 on %d cores: %.3f s per step" % (n, workers, med))
    return dict(points=out, host=host_info())


def cpu_baseline(scen, warm=1, steps=2):
    import numpy as np
    from oracle import Oracle
    o = Oracle(scen)
    o.step(warm)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return dict(value=round(scen.grid.npts * steps / dt, 1), unit="grid-point updates/s",
                cores=o.workers, kind="oracle",
                sample="FP64 NumPy/SciPy oracle, %d timed steps (after %d warm-up) of the same "
                       "256^3 tissue workload; %.1f s" % (steps, warm, dt),
                host=host_info())


def serving_bench(n_requests, rate=20.0, seed=0):
    """Continuous batching vs one-at-a-time FIFO on the same Poisson trace,
    then both again at a sustainable rate (70 % of the measured batched
    capacity)."""
    from paper_1408_4675_amd import scenarios as sc
    from paper_1408_4675_amd.serving import Server, run_fifo, summarize
    log("building the serving trace (%d requests, %.0f/s)" % (n_requests, rate))
    reqs = sc.serving_trace(seed=seed, n_requests=n_requests, rate=rate, medium_pool=2)
    out = dict(metric="serving latency and throughput (Poisson trace, 64^3-256^3 tissue)",
               trace=dict(requests=n_requests, rate_per_s=rate, seed=seed,
                          sizes=list(sc.SERVING_SIZES), steps="300-1500",
                          offered_point_updates_per_s=rate * float(np.mean(
                              [r.scenario.grid.npts * r.scenario.steps for r in reqs]))))
    def progress(tag):
        return lambda r: log("%s: request %d done (%.1f s after arrival)" % (tag, r.rid, r.latency))

    log("batched")
    srv = Server(max_active=8, chunk_steps=64)
    out["batched"] = summarize(srv.run(reqs, on_done=progress("batched")))
    out["batched"]["peak_active"] = srv.peak_active
    log("batched: %s" % json.dumps(out["batched"]))
    log("fifo")
    out["fifo"] = summarize(run_fifo(reqs, on_done=progress("fifo")))
    log("fifo: %s" % json.dumps(out["fifo"]))
    cap = out["batched"]["point_updates_per_s"]
    work = float(np.mean([r.scenario.grid.npts * r.scenario.steps for r in reqs]))
    lam = 0.7 * cap / work
    log("sustainable rate %.2f/s" % lam)
    reqs2 = sc.serving_trace(seed=seed, n_requests=n_requests, rate=lam, medium_pool=2)
    out["sustainable_rate_per_s"] = lam
    srv2 = Server(max_active=8, chunk_steps=64)
    out["batched_at_sustainable"] = summarize(srv2.run(reqs2, on_done=progress("batched, sustainable")))
    log("batched at sustainable: %s" % json.dumps(out["batched_at_sustainable"]))
    out["fifo_at_sustainable"] = summarize(run_fifo(reqs2, on_done=progress("fifo, sustainable")))
    return out


def serving_summary(n_requests, rate=20.0, seed=0):
    """The latency half of the metric, measured in the default run: the
    first `n_requests` requests of the Poisson serving trace (20/s, 64^3-256^3
    tissue, 300-1500 steps) served with continuous batching and one at a time
    (FIFO), p50 / p99 latency from arrival to gathered result, and
    throughput."""
    from paper_1408_4675_amd import scenarios as sc
    from paper_1408_4675_amd.serving import Server, run_fifo, summarize
    log("serving: building %d requests" % n_requests)
    reqs = sc.serving_trace(seed=seed, n_requests=n_requests, rate=rate, medium_pool=2)
    done = lambda tag: (lambda r: log("serving %s: request %d done" % (tag, r.rid)))
    srv = Server(max_active=8, chunk_steps=64)
    b = summarize(srv.run(reqs, on_done=done("batched")))
    f = summarize(run_fifo(reqs, on_done=done("fifo")))
    keys = ("p50_latency_s", "p99_latency_s", "requests_per_s", "point_updates_per_s",
            "makespan_s")
    return dict(workload="first %d requests of the Poisson trace (seed %d, %.0f/s offered, "
                         "64^3-256^3 tissue, 300-1500 steps)" % (n_requests, seed, rate),
                batched={k: round(b[k], 4) for k in keys},
                fifo={k: round(f[k], 4) for k in keys},
                peak_active=srv.peak_active)


def adjoint_bench(checkpoint_every=50, fd_params=4):
    """Gradient of J = mean intensity in a 2 mm sphere at the focus minus the
    mean outside, with respect to the 64 element amplitudes and phases, on the
    128^3 tissue bowl (600 steps, intensity over the last 200).  Reports the
    forward and reverse wall times and a central-difference check of a few
    parameters through the float32 forward model."""
    from paper_1408_4675_amd import scenarios as sc
    from paper_1408_4675_amd.adjoint import focus_gradient, with_drive, _Run
    scen, focus = sc.adjoint_bowl(seed=0)
    w = sc.focal_weights(scen.grid, focus, 2e-3)
    rng = np.random.default_rng(1)
    ne = len(scen.source.amp)
    amp = rng.uniform(0.5e6, 1.5e6, ne)
    ph = rng.uniform(-np.pi, np.pi, ne)
    scen = with_drive(scen, amp, ph)
    log("adjoint: warm-up")
    focus_gradient(scen.replace(steps=60, sensor=sc.Sensor(record=sc.REC_INTENSITY,
                                                           record_start=41)), w, checkpoint_every)
    log("adjoint: gradient")
    out = focus_gradient(scen, w, checkpoint_every)
    steps = scen.steps
    res = dict(metric="focusing-objective gradient (128^3 tissue, 64 elements, 600 steps)",
               J=out["J"], steps=steps, checkpoint_every=checkpoint_every,
               forward_s=round(out["forward_s"], 4), backward_s=round(out["backward_s"], 4),
               forward_ms_per_step=round(out["forward_s"] / steps * 1e3, 4),
               backward_ms_per_step=round(out["backward_s"] / steps * 1e3, 4),
               grad_amp_norm=float(np.linalg.norm(out["grad_amp"])),
               grad_phase_norm=float(np.linalg.norm(out["grad_phase"])))
    # central differences through the float32 forward model
    checks = []
    pick = np.argsort(-np.abs(out["grad_amp"]))[: fd_params // 2]
    for e in pick:
        for kind in ("amp", "phase"):
            a2, p2 = amp.copy(), ph.copy()
            h = 1e-2 * amp[e] if kind == "amp" else 1e-2
            vals = []
            for sgn in (1, -1):
                if kind == "amp":
                    a2[e] = amp[e] + sgn * h
                else:
                    p2[e] = ph[e] + sgn * h
                r = _Run(with_drive(scen, a2, p2), w, checkpoint_every)
                vals.append(r.J)
                r.close()
            fd = (vals[0] - vals[1]) / (2 * h)
            g = out["grad_amp"][e] if kind == "amp" else out["grad_phase"][e]
            checks.append(dict(element=int(e), param=kind, adjoint=float(g), fd=float(fd),
                               rel_diff=float(abs(g - fd) / max(abs(fd), 1e-300))))
    res["fd_checks"] = checks
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-large", action="store_true", help="skip the 1024^3 item")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--large-steps", type=int, default=100)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving latency item")
    ap.add_argument("--serving-requests", type=int, default=30,
                    help="requests of the serving trace in the default run's latency item")
    ap.add_argument("--serving", type=int, default=0, metavar="N",
                    help="instead of the step benchmark, serve the first N requests of the "
                         "Poisson trace (20/s, 64^3-256^3 tissue) batched and one at a time")
    ap.add_argument("--cpu-scaling", action="store_true",
                    help="instead of the step benchmark, time the FP64 oracle at 64^3, 128^3 and "
                         "256^3 on all host cores and on one core")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the step benchmark, time the gradient of the focusing "
                         "objective (128^3 tissue, 64-element bowl, 600 steps)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.cpu_scaling:
        # host only: no GPU needed
        print(json.dumps(dict(metric="FP64 oracle grid-point updates/s on the host",
                              oracle=cpu_scaling(), paper_context=PAPER_CONTEXT)), flush=True)
        return

    import torch
    from paper_1408_4675_amd import scenarios as sc
    from paper_1408_4675_amd import _abi
    _abi.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.adjoint:
        print(json.dumps(adjoint_bench()), flush=True)
        return
    if args.serving:
        print(json.dumps(serving_bench(args.serving)), flush=True)
        return

    log("building 256^3 tissue workload")
    scen = sc.tissue_bowl(seed=0, n=256, steps=args.steps)
    npts = scen.grid.npts
    log("timing %d steps after %d warm-up" % (args.steps, args.warmup))
    secs, psecs, stats = time_workload(scen, args.steps, args.warmup)
    ms_per_step = secs / args.steps * 1e3
    value = npts * args.steps / secs
    dom, roof, per_class = roofline(stats, npts)
    step_bytes = pass_model_bytes(stats) / args.steps
    out = dict(
        metric="grid-point updates/s (256^3 heterogeneous nonlinear absorbing step, FP32)",
        value=round(value, 1), unit="grid-point updates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(ms_per_step, 4), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="tissue_bowl_256: 256^3 layered tissue + inclusions (seed 0), "
                             "1 MHz 5 MPa bowl R15/aperture 18 mm, PML 20, CFL 0.3, "
                             "p_max+p_rms at all points", grid=[256, 256, 256],
                    kernels_per_step=stats["kernels_per_step"],
                    fft_per_step=stats["fft_forward_per_step"] + stats["fft_inverse_per_step"]),
        roofline=roof,
        step_roofline=dict(pass_model_bytes_per_point=round(step_bytes / npts, 2),
                           achieved_gbs=round(step_bytes / (ms_per_step / 1e3) / 1e9, 1),
                           frac=round(step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                           # state u, rho r/w (48 B) + 4 medium maps (16 B) + 2 sensor
                           # accumulators r/w (16 B): what any scheme must move per step
                           compulsory_bytes_per_point=80,
                           compulsory_frac=round(80.0 * npts / (ms_per_step / 1e3) / 1e9
                                                 / HBM_PEAK_GBS, 4)),
        per_class=per_class,
        # the roofline and per-class durations come from a second region of the
        # same length, launched eagerly with HIP events around every kernel
        profiled_ms_per_step=round(psecs / args.steps * 1e3, 4),
    )
    log("measuring the device copy ceiling")
    out["copy_ceiling_gbs"] = copy_ceiling()
    if not args.no_large:
        try:
            log("building 1024^3 water workload")
            big = sc.water_bowl_large(n=1024, steps=args.large_steps)
            warm = min(20, args.large_steps)
            log("timing 1024^3: %d steps after %d warm-up" % (args.large_steps, warm))
            bsecs, bpsecs, bstats = time_workload(big, args.large_steps, warm)
            bms = bsecs / args.large_steps * 1e3
            bdom, broof, bper = roofline(bstats, big.grid.npts)
            bstep = pass_model_bytes(bstats) / args.large_steps
            out["large"] = dict(workload="water_bowl_1024: 1024^3 homogeneous water, 3 MHz 2 MPa "
                                         "bowl, PML 20, one focal sensor",
                                value=round(big.grid.npts * args.large_steps / bsecs, 1),
                                unit="grid-point updates/s", ms_per_step=round(bms, 3),
                                profiled_ms_per_step=round(bpsecs / args.large_steps * 1e3, 3),
                                steps=args.large_steps, roofline=broof,
                                step_roofline=dict(
                                    pass_model_bytes_per_point=round(bstep / big.grid.npts, 2),
                                    achieved_gbs=round(bstep / (bms / 1e3) / 1e9, 1),
                                    frac=round(bstep / (bms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)),
                                per_class=bper)
        except Exception as e:   # report, but keep the headline line
            out["large"] = dict(error=str(e))
    if not args.no_serving:
        try:
            out["serving"] = serving_summary(args.serving_requests)
        except Exception as e:   # report, but keep the headline line
            out["serving"] = dict(error=str(e))
    out["paper_context"] = PAPER_CONTEXT
    if not args.no_cpu:
        log("timing the CPU oracle baseline")
        # about 12 s of FP64 work on a 16-core host (1.4 s per step)
        out["cpu_baseline"] = cpu_baseline(sc.tissue_bowl(seed=0, n=256, steps=9), warm=1, steps=8)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
