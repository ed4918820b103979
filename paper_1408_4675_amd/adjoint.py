"""Gradients of the focusing objective with respect to the source drive.

J = sum_x w(x) I(x), I the time-mean intensity over the recorded steps, is
differentiated through the float32 time stepping by the library's reverse-mode
step (kw_adjoint_*).  The forward run keeps a snapshot (kw_save) every
`checkpoint_every` steps; the reverse sweep walks the segments backwards,
restores each segment's snapshot, re-runs the segment forward writing a step
record (kw_adjoint_record: the divergence, the density components and the
pressure spectrum of the step) for every step, and applies the reverse steps
from the last to the first, each reading its record.  Device memory: one
snapshot per segment plus one record (7 fields) per step of a segment.

`FocusObjective` wraps this as a torch.autograd.Function of the element
amplitudes and phases.  This module only sequences library calls.
"""
from __future__ import annotations

import ctypes as C
import time
from typing import Optional

import numpy as np
import torch

from . import _abi as A
from .scenarios import Scenario, Source
from .simulation import Simulation


class Adjoint:
    """The reverse-mode state of one simulation (kw_adj)."""

    def __init__(self, sim: Simulation, weights, n_steps: int):
        self.lib = A.load()
        self.sim = sim
        self.n_steps = int(n_steps)
        w = np.ascontiguousarray(np.asarray(weights, np.float32).reshape(-1))
        if w.size != sim.npts:
            raise ValueError("weights have %d values, the grid has %d" % (w.size, sim.npts))
        nb = self.lib.kw_adjoint_workspace_size(sim.handle, self.n_steps)
        if nb == 0:
            raise A.KwError(A.KW_EINVAL, self.lib.kw_last_error().decode())
        self.workspace = torch.empty(int(nb), dtype=torch.uint8, device=sim.device)
        # ordered before the simulation's stream; close() synchronises that
        # stream before the workspace goes back to torch (no record_stream:
        # the simulation may own its stream and destroy it on close)
        sim.stream.wait_stream(torch.cuda.current_stream(sim.device))
        h = C.c_void_p()
        A.check(self.lib.kw_adjoint_create(sim.handle, w.ctypes.data_as(C.POINTER(C.c_float)),
                                           self.n_steps, C.c_void_p(self.workspace.data_ptr()),
                                           C.c_size_t(nb), C.byref(h)))
        self.handle = h

    def objective(self) -> float:
        J = C.c_double()
        A.check(self.lib.kw_adjoint_objective(self.handle, C.byref(J)))
        return J.value

    def step(self, n: int):
        A.check(self.lib.kw_adjoint_step(self.handle, int(n)))

    def record_bytes(self) -> int:
        return int(self.lib.kw_adjoint_record_bytes(self.handle))

    def new_record(self) -> torch.Tensor:
        """A device buffer for one step record, ordered before the simulation's stream."""
        r = torch.empty(self.record_bytes(), dtype=torch.uint8, device=self.sim.device)
        self.sim.stream.wait_stream(torch.cuda.current_stream(self.sim.device))
        return r

    def record(self, rec: torch.Tensor):
        """Advance the simulation one step, writing that step's record to rec."""
        A.check(self.lib.kw_adjoint_record(self.handle, C.c_void_p(rec.data_ptr()),
                                           C.c_size_t(rec.numel())))

    def step_record(self, n: int, rec: torch.Tensor):
        """Reverse step n from the record of forward step n."""
        A.check(self.lib.kw_adjoint_step_record(self.handle, int(n), C.c_void_p(rec.data_ptr()),
                                                C.c_size_t(rec.numel())))

    def source_gradient(self) -> np.ndarray:
        ne = len(self.sim.scenario.source.amp)
        out = np.zeros((self.n_steps, ne), np.float64)
        A.check(self.lib.kw_adjoint_source_gradient(
            self.handle, out.ctypes.data_as(C.POINTER(C.c_double)), C.c_size_t(out.nbytes)))
        return out

    def gradient(self):
        ne = len(self.sim.scenario.source.amp)
        ga = np.zeros(ne, np.float64)
        gp = np.zeros(ne, np.float64)
        A.check(self.lib.kw_adjoint_gradient(self.handle, ga.ctypes.data_as(C.POINTER(C.c_double)),
                                             gp.ctypes.data_as(C.POINTER(C.c_double))))
        return ga, gp

    def close(self):
        if getattr(self, "handle", None):
            self.lib.kw_adjoint_destroy(self.handle)     # synchronises the stream
            self.handle = None
        self.workspace = None


def with_drive(scen: Scenario, amp, phase) -> Scenario:
    src = scen.source
    return scen.replace(source=Source(index=src.index, element=src.element,
                                      amp=np.asarray(amp, np.float32),
                                      phase=np.asarray(phase, np.float32), freq=src.freq))


class _Run:
    """A forward run with checkpoints, ready for the reverse sweep."""

    def __init__(self, scen: Scenario, weights, checkpoint_every: int = 50,
                 device: str = "cuda"):
        self.scen = scen
        self.K = int(checkpoint_every)
        self.T = int(scen.steps)
        self.sim = Simulation(scen, device=device)
        self.adj = Adjoint(self.sim, weights, self.T)
        self.records = [self.adj.new_record() for _ in range(min(self.K, self.T))]
        self.ckpt = {}
        t0 = time.perf_counter()
        for n0 in range(0, self.T, self.K):
            self.ckpt[n0] = self.sim.save(device=True)
            self.sim.step(min(self.K, self.T - n0))
        self.J = self.adj.objective()
        self.forward_s = time.perf_counter() - t0

    def backward(self):
        sim, adj = self.sim, self.adj
        t0 = time.perf_counter()
        for n0 in sorted(self.ckpt, reverse=True):
            n1 = min(n0 + self.K, self.T)
            sim.load(self.ckpt[n0])
            for j in range(n1 - n0):
                adj.record(self.records[j])
            for n in range(n1 - 1, n0 - 1, -1):
                adj.step_record(n, self.records[n - n0])
        ga, gp = adj.gradient()
        sim.synchronize()
        self.backward_s = time.perf_counter() - t0
        return ga, gp

    def close(self):
        self.adj.close()
        self.records = None
        self.sim.close()


def focus_gradient(scen: Scenario, weights, checkpoint_every: int = 50,
                   device: str = "cuda") -> dict:
    """J and its gradient with respect to the amplitudes and phases of the
    source elements, plus the wall time of both sweeps."""
    run = _Run(scen, weights, checkpoint_every, device)
    try:
        ga, gp = run.backward()
        return dict(J=run.J, grad_amp=ga, grad_phase=gp, forward_s=run.forward_s,
                    backward_s=run.backward_s, source_gradient=run.adj.source_gradient())
    finally:
        run.close()


class FocusObjective(torch.autograd.Function):
    """J(amp, phase) for a fixed medium, geometry and weight map; amp and
    phase are float64 tensors of one value per element."""

    @staticmethod
    def forward(ctx, amp, phase, scen: Scenario, weights, checkpoint_every: int = 50):
        s = with_drive(scen, amp.detach().cpu().numpy(), phase.detach().cpu().numpy())
        run = _Run(s, weights, checkpoint_every)
        ctx.run = run
        return torch.tensor(run.J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        run = ctx.run
        try:
            ga, gp = run.backward()
        finally:
            run.close()
        g = float(gJ)
        return (torch.from_numpy(ga * g), torch.from_numpy(gp * g), None, None, None)
