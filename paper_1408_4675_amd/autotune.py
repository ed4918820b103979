"""FFT schedule autotuner.

For each axis of a grid it times candidate radix schedules (and, for the
column passes, column-tile widths; for the x rows, rows per block) with the
library's per-kernel HIP-event profiling, keeps the fastest, and caches the
choice as JSON keyed by device architecture, axis kind and transform length.
`Simulation` applies cached choices automatically; without a cache the
library's built-in defaults are used.  This plays the role that FFT planning
by measurement plays in the paper's cluster code (Section 3.4), but the search
space is this library's own: radix factorisations 2/3/4/5/8/16(/32) and tile
shapes of the LDS-staged passes.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

CACHE_ENV = "KW_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kw_tune.json")

# kernel classes whose time depends on each axis' schedule
AXIS_CLASSES = {0: ("xvel", "xden", "xeos"),
                1: ("ypass_fwd", "ypass_inv"),
                2: ("zfused_grad", "zfused_div", "zfused_abs")}


def cache_path() -> str:
    return os.environ.get(CACHE_ENV, DEFAULT_CACHE)


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache() -> Dict:
    p = cache_path()
    if os.path.exists(p):
        try:
            with open(p) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}
    return {}


def save_cache(d: Dict):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def key(axis: int, n: int, arch: Optional[str] = None) -> str:
    return "%s|%s|%d" % (arch or _arch(), "xyz"[axis], n)


SHIPPED_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


def shipped_table(arch: Optional[str] = None) -> Dict:
    """Choices measured for this package on `arch` and shipped with it."""
    p = os.path.join(SHIPPED_DIR, "%s.json" % (arch or _arch()))
    if os.path.exists(p):
        with open(p) as fh:
            return json.load(fh)
    return {}


def lengths(grid) -> Tuple[int, int, int]:
    """Transform length per axis: nx/2 for the packed x rows, ny, nz."""
    return (grid.nx // 2, grid.ny, grid.nz)


def _factorisations(n: int, radices: Sequence[int], max_passes: int = 4) -> List[List[int]]:
    out = []

    def rec(m, cur):
        if m == 1:
            out.append(list(cur))
            return
        if len(cur) >= max_passes:
            return
        for r in radices:
            if m % r == 0 and (not cur or r <= cur[-1]):
                cur.append(r)
                rec(m // r, cur)
                cur.pop()
    rec(n, [])
    return out


def candidates(axis: int, n: int) -> List[Tuple[List[int], int]]:
    """(radix schedule, tile) pairs worth timing for one axis."""
    pow2 = n & (n - 1) == 0
    if pow2:
        scheds = _factorisations(n, (16, 8, 4, 2), 4)
        # keep the shortest schedules (at most one pass more than the minimum)
        mn = min(len(s) for s in scheds)
        scheds = [s for s in scheds if len(s) <= mn + 1]
        if n >= 32:
            # the 32-wide fixed engine: radix-32 passes only
            scheds += _factorisations(n, (32,), 3)
        # the four-wide fixed engine (radices up to 4: more passes, fewer
        # registers per thread)
        four = _factorisations(n, (4, 2), 8)
        if four:
            mn4 = min(len(s) for s in four)
            scheds += [s for s in four if len(s) == mn4 and s not in scheds][:1]
    else:
        scheds = _factorisations(n, (16, 15, 12, 10, 8, 6, 5, 4, 3, 2), 3)
        mn = min(len(s) for s in scheds)
        scheds = [s for s in scheds if len(s) == mn][:6]
        # the mixed-radix fixed engine (12 or 20 elements per thread): the
        # shortest schedules of radices that divide its width
        for w in (12, 20):
            if n % w == 0:
                mixed = _factorisations(n, [q for q in (20, 12, 10, 6, 5, 4, 3, 2) if w % q == 0], 4)
                if mixed:
                    mnm = min(len(s) for s in mixed)
                    scheds += [s for s in mixed if len(s) == mnm and s not in scheds][:3]
    tiles = (0, 4, 8, 16, 32) if axis == 0 else (0, 8, 16, 32)
    return [(s, t) for s, t in itertools.product(scheds, tiles)]


def _time_axis(scen, axis: int, sched: List[int], tile: int, steps: int) -> Optional[float]:
    from . import _abi as A
    from .simulation import Simulation
    try:
        sim = Simulation(scen, tune=False)
        sim.set_plan(axis, sched, tile)
    except A.KwError:
        return None
    sim.step(2)
    sim.synchronize()
    sim.stats()
    sim.profile(True)
    base = sim.stats()["classes"]
    sim.step(steps)
    st = sim.stats()["classes"]
    sim.profile(False)
    sim.close()
    return sum(st[c]["ms"] - base[c]["ms"] for c in AXIS_CLASSES[axis]) / steps


def tune(scen, axes=(0, 1, 2), steps: int = 4, verbose: bool = True, save: bool = True) -> Dict:
    """Time every candidate schedule for the requested axes of `scen` and
    record the fastest in the cache.  Returns {axis: (schedule, tile, ms)}."""
    cache = load_cache()
    arch = _arch()
    result = {}
    for axis in axes:
        n = lengths(scen.grid)[axis]
        best = None
        for sched, tile in candidates(axis, n):
            ms = _time_axis(scen, axis, sched, tile, steps)
            if ms is None:
                continue
            if verbose:
                print("tune axis %d n=%d %-14s tile %2d: %.4f ms/step" % (axis, n, sched, tile, ms),
                      flush=True)
            if best is None or ms < best[2]:
                best = (sched, tile, ms)
        if best is not None:
            result[axis] = best
            cache[key(axis, n, arch)] = dict(radices=best[0], tile=best[1], ms=best[2])
    if save:
        save_cache(cache)
    return result


def lookup(grid) -> Dict[int, Tuple[List[int], int]]:
    """Choices for the axes of `grid`: the user's cache first, then the table
    shipped with the package ({} when neither has an entry)."""
    arch = _arch()
    tables = (load_cache(), shipped_table(arch))
    out = {}
    for axis, n in enumerate(lengths(grid)):
        for tab in tables:
            e = tab.get(key(axis, n, arch))
            if e:
                out[axis] = (list(e["radices"]), int(e.get("tile", 0)))
                break
    return out


def tune_table(sizes, steps: int = 3, out: Optional[str] = None, verbose: bool = True) -> Dict:
    """Tune every axis for each cubic size in `sizes` (for lengths above 256
    on a grid whose other two axes are 64 points, one axis at a time) and
    return {key: choice}; with `out`, also write it as JSON (the format of the
    shipped tables)."""
    from . import scenarios as sc
    arch = _arch()
    table = {}
    for n in sizes:
        if n <= 256:
            jobs = [(sc.small_case(n, n, n, seed=0, steps=8), (0, 1, 2))]
        else:
            jobs = []
            for axis in range(3):
                shape = [64, 64, 64]
                shape[axis] = n
                jobs.append((sc.small_case(*shape, seed=0, steps=8), (axis,)))
        for scen, axes in jobs:
            res = tune(scen, axes=axes, steps=steps, verbose=verbose, save=False)
            for axis, (sched, tile, ms) in res.items():
                table[key(axis, lengths(scen.grid)[axis], arch)] = dict(radices=sched, tile=tile,
                                                                         ms=round(ms, 5))
            if verbose:
                print("tuned n=%d axes %s" % (n, axes), flush=True)
    if out:
        with open(out, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    return table


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_1408_4675_amd.autotune")
    ap.add_argument("--sizes", type=int, nargs="+", default=[64, 96, 128, 160, 192, 256, 1024])
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--out", default=None, help="write the table here (JSON)")
    a = ap.parse_args()
    tune_table(a.sizes, a.steps, a.out)
