"""Serving loop: many independent simulations on one GPU.

Requests (a Scenario and an arrival time) are admitted while the sum of their
device footprints (kw_workspace_size, exact) stays within an HBM budget and
fewer than `max_active` run.  Every admitted simulation keeps its fields
resident in its own workspace and runs on a HIP stream of its own, advanced in
chunks of `chunk_steps` steps (captured HIP graphs); a chunk is enqueued as
soon as the previous one of that simulation has finished, so simulations of
different sizes interleave on the GPU (continuous batching).

Set-up is split in two.  The host part (kw_prepare: validation, FFT plans,
float64 tables and medium maps -- the bulk of the set-up time at 256^3) runs in
a pool of worker threads as soon as a request arrives, a few requests ahead of
admission; it makes no HIP call.  The device part (workspace, stream, upload)
and every other call that touches the GPU run in the scheduling thread only.
Each result is computed by exactly the same kernels, in the same order, as
when the request runs alone, so it is bit-for-bit the same.

`run_fifo` is the baseline: one request at a time, in arrival order.

All device work goes through the C ABI (Simulation); this module only
schedules.
"""
from __future__ import annotations

import concurrent.futures as cf
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A
from .scenarios import REC_P_MAX, REC_P_RMS, Request
from .simulation import Prepared, Simulation, workspace_size


@dataclass
class Result:
    rid: int
    n: int                     # grid points
    steps: int
    arrival: float             # seconds after the start of the run
    start: float               # admission time
    finish: float              # outputs gathered
    outputs: Dict[int, np.ndarray] = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def _gather(sim: Simulation, record: int, keep: bool) -> Dict[int, np.ndarray]:
    out = {}
    for what in (REC_P_MAX, REC_P_RMS):
        if record & what:
            v = sim.gather(what, device=False)
            if keep:
                out[what] = v
    return out


@dataclass
class _Active:
    req: Request
    sim: Simulation
    left: int
    start: float
    event: Optional[torch.cuda.Event] = None


class Server:
    """Continuous-batching scheduler over one GPU."""

    def __init__(self, budget_bytes: Optional[int] = None, max_active: int = 8,
                 chunk_steps: int = 64, keep_outputs: bool = False, device: str = "cuda",
                 prepare_workers: int = 2, prepare_ahead: Optional[int] = None):
        self.device = torch.device(device)
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            budget_bytes = int(free * 0.8)
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.chunk = chunk_steps
        self.keep = keep_outputs
        self.workers = max(1, int(prepare_workers))
        # arrived requests whose host preparation may be under way or done but
        # not yet admitted (each holds its tables and maps in host memory)
        self.ahead = max(1, int(prepare_ahead if prepare_ahead is not None else max_active))
        self.peak_used = 0             # largest sum of admitted footprints seen
        self.peak_active = 0           # largest number of simulations admitted at once

    def run(self, requests: Sequence[Request], on_done: Optional[Callable] = None) -> List[Result]:
        A.load()
        reqs = sorted(requests, key=lambda r: r.arrival)
        foot = {r.rid: workspace_size(r.scenario) for r in reqs}
        for r in reqs:
            if foot[r.rid] > self.budget:
                raise ValueError("request %d needs %d bytes, budget is %d"
                                 % (r.rid, foot[r.rid], self.budget))
        pending = list(reqs)                 # not admitted, in arrival order
        prepared: Dict[int, cf.Future] = {}  # host preparation of pending requests
        active: List[_Active] = []
        results: List[Result] = []
        used = 0
        pool = cf.ThreadPoolExecutor(max_workers=self.workers)
        t0 = time.perf_counter()
        try:
            while pending or active:
                now = time.perf_counter() - t0
                # host preparation of the first arrived requests (no device calls)
                for r in pending[: self.ahead]:
                    if r.arrival > now:
                        break
                    if r.rid not in prepared:
                        prepared[r.rid] = pool.submit(Prepared, r.scenario)
                # admission: arrived and prepared, a slot free, footprint within
                # budget, strictly in arrival order
                while (pending and pending[0].rid in prepared and prepared[pending[0].rid].done()
                       and len(active) < self.max_active
                       and used + foot[pending[0].rid] <= self.budget):
                    r = pending.pop(0)
                    prep = prepared.pop(r.rid).result()
                    used += foot[r.rid]
                    try:
                        active.append(self._create(r, now, prep))
                    finally:
                        prep.close()
                    self.peak_used = max(self.peak_used, used)
                    self.peak_active = max(self.peak_active, len(active))
                progressed = False
                for a in list(active):
                    if a.event is not None and not a.event.query():
                        continue
                    progressed = True
                    if a.left > 0:
                        n = min(self.chunk, a.left)
                        a.sim.step(n)
                        a.left -= n
                        a.event = torch.cuda.Event()
                        a.event.record(a.sim.stream)
                        continue
                    outs = _gather(a.sim, a.req.scenario.sensor.record, self.keep)
                    fin = time.perf_counter() - t0
                    res = Result(a.req.rid, a.req.scenario.grid.npts, a.req.scenario.steps,
                                 a.req.arrival, a.start, fin, outs)
                    a.sim.close()
                    active.remove(a)
                    used -= foot[a.req.rid]
                    results.append(res)
                    if on_done:
                        on_done(res)
                if not progressed:
                    # nothing to issue: wait briefly for an arrival, a preparation
                    # or a chunk to end
                    nxt = pending[0].arrival - (time.perf_counter() - t0) if pending else 1.0
                    time.sleep(max(0.0, min(nxt, 2e-4)))
        finally:
            pool.shutdown(wait=True)
            for f in prepared.values():
                if f.done() and f.exception() is None:
                    f.result().close()
            for a in active:
                a.sim.close()
        return sorted(results, key=lambda r: r.rid)

    def _create(self, r: Request, now: float, prep: Optional[Prepared] = None) -> _Active:
        sim = Simulation(r.scenario, device=str(self.device), prepared=prep)
        return _Active(r, sim, r.scenario.steps, now)


def run_fifo(requests: Sequence[Request], keep_outputs: bool = False,
             device: str = "cuda", on_done: Optional[Callable] = None) -> List[Result]:
    """Baseline: one request at a time in arrival order (each waits for the
    previous one to finish)."""
    A.load()
    reqs = sorted(requests, key=lambda r: r.arrival)
    results = []
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        start = time.perf_counter() - t0
        sim = Simulation(r.scenario, device=device)
        sim.step(r.scenario.steps)
        outs = _gather(sim, r.scenario.sensor.record, keep_outputs)
        fin = time.perf_counter() - t0
        sim.close()
        results.append(Result(r.rid, r.scenario.grid.npts, r.scenario.steps, r.arrival, start,
                              fin, outs))
        if on_done:
            on_done(results[-1])
    return results


def summarize(results: Sequence[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    makespan = max(r.finish for r in results) - min(r.arrival for r in results)
    work = float(sum(r.n * r.steps for r in results))
    return dict(requests=len(results), p50_latency_s=float(np.percentile(lat, 50)),
                p99_latency_s=float(np.percentile(lat, 99)), mean_latency_s=float(lat.mean()),
                makespan_s=makespan, requests_per_s=len(results) / makespan,
                point_updates_per_s=work / makespan)
