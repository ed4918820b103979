"""Summaries of rocprofv3 runs of this library, and a plain copy kernel that
calibrates the HBM traffic counters.

    python -m paper_1408_4675_amd.profiling run --workload W [--steps K] [--warmup W0] [--eager]
        K steps of one workload on the GPU, for rocprofv3 to watch: W is
        tissue_bowl_N (N^3 layered tissue, bowl, all-point p_max / p_rms; N one
        of the serving sizes or 256) or water_bowl_1024 (1024^3 water, one
        focal sensor); captured graphs unless --eager
    python -m paper_1408_4675_amd.profiling copy [--mib N] [--reps K]
        a device-to-device copy of N MiB, K times (the reference kernel whose
        FETCH_SIZE / WRITE_SIZE give bytes-per-KiB scale factors)
    python -m paper_1408_4675_amd.profiling zcopy --out FILE.md
        build and run probes/zcol_copy.hip, a copy with the z passes' HBM
        access pattern (column tiles of packed spectra, no transform), and
        write its table: the bandwidth ceiling of a z pass for a tile width
    python -m paper_1408_4675_amd.profiling stats DIR --out FILE.md --title T --command C [--min-us U]
        turn the kernel_stats.csv that `rocprofv3 --kernel-trace --stats
        --output-format csv` wrote under DIR into a short Markdown table (with
        --min-us, from kernel_trace.csv, dispatches of at least U us only)
    python -m paper_1408_4675_amd.profiling traffic --fetch DIR --write DIR
            --copy-fetch DIR --copy-write DIR --copy-mib N --points P --out FILE.json --command C
        mean FETCH_SIZE and WRITE_SIZE per dispatch of every kernel class,
        scaled by what the counters read for the copy kernel, as JSON with the
        hash of the kernel sources they were taken on

Nothing here computes any part of the solver.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from typing import Dict, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# kernel name fragment -> class name reported by kw_stats
CLASS_OF = (("kw_ypass", None), ("kw_zfused", None), ("kw_xvel", "xvel"), ("kw_xden", "xden"),
            ("kw_xeos", "xeos"), ("kw_xfwd", "xfwd"), ("kw_xinv", "xinv"),
            ("kw_finalize", "finalize"), ("kw_fill", "fill"),
            ("kw_adjx_eos", "adjx_eos"), ("kw_adjx_den", "adjx_den"), ("kw_adjx_vel", "adjx_vel"),
            ("kw_adjx_sum", "adjx_sum"), ("kw_adj_src", "adj_src"), ("kw_adj_", "adj_setup"))


def kernel_source_hash() -> str:
    """Hash of every kernel source file; a traffic table is valid only for
    the sources it was measured on."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_class(name: str) -> Optional[str]:
    """Class of a demangled kernel name (None for kernels of other code)."""
    # (the engine is the first template argument, itself a template: the
    # direction flag is the first argument after it)
    m = re.search(r"kw_ypass<(?:kw::)?Eng\w+<[^<>]*>, (true|false)(, \d+)?>", name)
    if m:
        return "ypass_inv" if m.group(1) == "true" else "ypass_fwd"
    m = re.search(r"kw_zfused<.*?>, (\d)(, \d+)?(, (true|false))?>", name)
    if m:
        return {"0": "zfused_grad", "1": "zfused_div", "2": "zfused_abs",
                "3": "zfused_divt", "4": "zfused_gradt",
                "5": "zfused_abs"}.get(m.group(1), "zfused")   # 5: merged absorption
    for frag, cls in CLASS_OF:
        if cls and frag in name:
            return cls
    if "copy" in name.lower() or "elementwise" in name.lower():
        return "copy"
    return None


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return hits[-1]


def _col(row: Dict[str, str], *names: str) -> str:
    for n in names:
        if n in row:
            return row[n]
    raise KeyError("none of %s in %s" % (names, list(row)))


def read_kernel_stats(d: str) -> List[Dict]:
    with open(_find(d, "kernel_stats.csv")) as fh:
        rows = list(csv.DictReader(fh))
    out = []
    for r in rows:
        out.append(dict(name=_col(r, "Name", "KernelName", "Kernel_Name"),
                        calls=int(_col(r, "Calls")),
                        total_ns=float(_col(r, "TotalDurationNs", "Total_Duration_ns")),
                        avg_ns=float(_col(r, "AverageNs", "Average_ns")),
                        pct=float(_col(r, "Percentage"))))
    out.sort(key=lambda r: -r["total_ns"])
    return out


def read_kernel_trace(d: str, min_us: float) -> List[Dict]:
    """Per kernel name, calls and durations of the dispatches in
    kernel_trace.csv that lasted at least `min_us` microseconds."""
    with open(_find(d, "kernel_trace.csv")) as fh:
        rows = list(csv.DictReader(fh))
    per: Dict[str, List[float]] = {}
    for r in rows:
        ns = float(_col(r, "End_Timestamp")) - float(_col(r, "Start_Timestamp"))
        if ns >= min_us * 1e3:
            per.setdefault(_col(r, "Kernel_Name"), []).append(ns)
    tot = sum(sum(v) for v in per.values()) or 1.0
    out = [dict(name=k, calls=len(v), total_ns=sum(v), avg_ns=sum(v) / len(v),
                pct=100.0 * sum(v) / tot) for k, v in per.items()]
    out.sort(key=lambda r: -r["total_ns"])
    return out


def stats_markdown(d: str, title: str, command: str, min_us: float = 0.0) -> str:
    if min_us > 0:
        rows = read_kernel_trace(d, min_us)
        source = ("rocprofv3 kernel_trace.csv, dispatches of at least %g us only (this "
                  "selects the large workload's launches)" % min_us)
    else:
        rows = read_kernel_stats(d)
        source = "rocprofv3 kernel_stats.csv"
    lines = ["# %s" % title, "", "Command (from the repository root, on one MI355X; "
             "R is the repository root):", "", "    " + command, "",
             "Durations in microseconds, from %s." % source, "",
             "| kernel | class | calls | total us | average us | % |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| %s | %s | %d | %.1f | %.2f | %.1f |" % (
            r["name"].replace("|", "/"), kernel_class(r["name"]) or "-", r["calls"],
            r["total_ns"] / 1e3, r["avg_ns"] / 1e3, r["pct"]))
    per = {}
    for r in rows:
        c = kernel_class(r["name"])
        if c:
            e = per.setdefault(c, [0, 0.0])
            e[0] += r["calls"]
            e[1] += r["total_ns"]
    lines += ["", "Per class (average launch duration, us):", "",
              "| class | launches | average us |", "|---|---|---|"]
    for c, (n, ns) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        lines.append("| %s | %d | %.2f |" % (c, n, ns / n / 1e3))
    return "\n".join(lines) + "\n"


def read_counter(d: str, counter: str) -> Dict[str, List[float]]:
    """Per kernel class, the list of `counter` values (one per dispatch)."""
    with open(_find(d, "counter_collection.csv")) as fh:
        rows = list(csv.DictReader(fh))
    per: Dict[str, Dict[str, float]] = {}
    for r in rows:
        if _col(r, "Counter_Name", "Counter-Name") != counter:
            continue
        name = _col(r, "Kernel_Name", "Kernel-Name", "KernelName")
        disp = _col(r, "Dispatch_Id", "Dispatch-Id", "Correlation_Id")
        c = kernel_class(name)
        if c is None:
            continue
        # one row per dispatch (and per dimension instance: summed)
        per.setdefault(c, {}).setdefault(disp, 0.0)
        per[c][disp] += float(_col(r, "Counter_Value", "Counter-Value"))
    return {c: list(v.values()) for c, v in per.items()}


def _mean(x: List[float]) -> float:
    return sum(x) / len(x)


def traffic_table(fetch: str, write: str, copy_fetch: str, copy_write: str,
                  copy_mib: float) -> Dict:
    copy_bytes = copy_mib * 2 ** 20
    cf = read_counter(copy_fetch, "FETCH_SIZE")["copy"]
    cw = read_counter(copy_write, "WRITE_SIZE")["copy"]
    # the largest dispatches are the calibration copies (smaller ones are set-up)
    f_kib = max(cf)
    w_kib = max(cw)
    f_scale = copy_bytes / f_kib        # bytes per counter KiB
    w_scale = copy_bytes / w_kib
    kf = read_counter(fetch, "FETCH_SIZE")
    kw = read_counter(write, "WRITE_SIZE")
    kernels = {}
    for c in sorted(set(kf) & set(kw)):
        if c == "copy":
            continue
        fb = _mean(kf[c]) * f_scale
        wb = _mean(kw[c]) * w_scale
        kernels[c] = dict(fetch_bytes_per_launch=fb, write_bytes_per_launch=wb,
                          hbm_bytes_per_launch=fb + wb, dispatches=len(kf[c]))
    return dict(source_hash=kernel_source_hash(), copy_mib=copy_mib,
                copy_fetch_kib=f_kib, copy_write_kib=w_kib,
                fetch_scale_bytes_per_kib=f_scale, write_scale_bytes_per_kib=w_scale,
                kernels=kernels)


def copy_probe(mib: int, reps: int):
    import torch
    n = mib * 2 ** 20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d MiB %d times" % (mib, reps), flush=True)


def zcopy_probe(out: str, command: str):
    import shutil
    import subprocess
    import tempfile
    from . import build as B
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "probes", "zcol_copy.hip")
    with tempfile.TemporaryDirectory(prefix="kwprobe_") as tmp:
        exe = os.path.join(tmp, "zcol_copy")
        subprocess.run([B._hipcc(), "--offload-arch=" + B.ARCH, "-O3"] + B.DEVICE_FLAGS
                       + [src, "-o", exe], check=True)
        r = subprocess.run([exe], stdout=subprocess.PIPE, text=True, check=True)
    print(r.stdout, flush=True)
    with open(out, "w") as fh:
        fh.write("# Column-tile copy: the HBM ceiling of the z passes' access pattern\n\n")
        fh.write("Command (from the repository root, on one MI355X):\n\n    %s\n\n" % command)
        fh.write("A block copies a tile of adjacent columns of a field of packed spectra\n"
                 "(loads first, then stores; 'exchange' adds one LDS round trip with\n"
                 "barriers); bytes per row is the contiguous run a tile reads and writes\n"
                 "in each z plane.  TB/s counts the bytes read and written.\n\n")
        fh.write(r.stdout)
    print("wrote", out)


def run_workload(name: str, steps: int, warmup: int, eager: bool):
    import time
    import torch
    from . import scenarios as sc
    from .simulation import Simulation
    if name == "adjoint_bowl_128":
        # forward run with checkpoints every 50 steps, then the reverse sweep
        from .adjoint import _Run
        scen, focus = sc.adjoint_bowl(seed=0, steps=steps)
        w = sc.focal_weights(scen.grid, focus, 2e-3)
        r = _Run(scen, w, 50)
        r.backward()
        print("%s: %d steps, forward %.4f ms per step, reverse sweep %.4f ms per step" % (
            name, steps, r.forward_s / steps * 1e3, r.backward_s / steps * 1e3), flush=True)
        r.close()
        torch.cuda.synchronize()
        return
    if name.startswith("tissue_bowl_"):
        scen = sc.tissue_bowl(seed=0, n=int(name.split("_")[-1]), steps=steps)
    elif name == "water_bowl_1024":
        scen = sc.water_bowl_large(n=1024, steps=steps)
    else:
        raise SystemExit("unknown workload %s" % name)
    print("workload %s built" % name, flush=True)
    sim = Simulation(scen, graph_steps=0 if eager else None)
    sim.step(warmup)
    sim.synchronize()
    print("warm-up done", flush=True)
    t0 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    dt = time.perf_counter() - t0
    st = sim.stats()
    sim.close()
    torch.cuda.synchronize()
    print("%s: %d steps, %.4f ms per step, nonfinite step %d" % (
        name, steps, dt / steps * 1e3, st["nonfinite_step"]), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1408_4675_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("run")
    p.add_argument("--workload", required=True)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--eager", action="store_true")
    p = sub.add_parser("copy")
    p.add_argument("--mib", type=int, default=1024)
    p.add_argument("--reps", type=int, default=5)
    p = sub.add_parser("zcopy")
    p.add_argument("--out", required=True)
    p = sub.add_parser("stats")
    p.add_argument("dir")
    p.add_argument("--out", required=True)
    p.add_argument("--title", required=True)
    p.add_argument("--command", required=True)
    p.add_argument("--min-us", type=float, default=0.0,
                   help="summarise only dispatches at least this long (from kernel_trace.csv)")
    p = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "out", "command"):
        p.add_argument("--" + k, required=True)
    p.add_argument("--copy-mib", type=float, default=1024)
    p.add_argument("--points", type=int, required=True,
                   help="grid points of the profiled workload (the table applies to that grid only)")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run_workload(a.workload, a.steps, a.warmup, a.eager)
    elif a.cmd == "copy":
        copy_probe(a.mib, a.reps)
    elif a.cmd == "zcopy":
        zcopy_probe(a.out, "python -m paper_1408_4675_amd.profiling zcopy --out " + a.out)
    elif a.cmd == "stats":
        with open(a.out, "w") as fh:
            fh.write(stats_markdown(a.dir, a.title, a.command, a.min_us))
        print("wrote", a.out)
    else:
        d = traffic_table(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_mib)
        d["command"] = a.command
        d["points"] = a.points
        with open(a.out, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        print(json.dumps(d["kernels"], indent=1))


if __name__ == "__main__":
    sys.exit(main())
