"""Python front end of the HIP solver: PyTorch supplies the device workspace
and the stream, libkw.so does all the work.

    sim = Simulation(scenario)           # kw_create
    sim.step(200)                        # kw_step (asynchronous)
    p_max = sim.gather(REC_P_MAX)        # kw_gather -> torch tensor on the GPU
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch

from . import _abi as A
from .scenarios import Scenario

_P = C.POINTER


def _fptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_P(C.c_float))


def _map_or_scalar(v, n):
    """(pointer-keeper array or None, scalar)"""
    if np.isscalar(v) or np.ndim(v) == 0:
        return None, float(v)
    a = np.ascontiguousarray(np.asarray(v, np.float32).reshape(-1))
    if a.size != n:
        raise ValueError("medium map has %d values, grid has %d" % (a.size, n))
    return a, 0.0


class _Marshalled:
    """ctypes structs for one scenario; keeps the numpy buffers alive."""

    def __init__(self, sc: Scenario):
        g, m = sc.grid, sc.medium
        n = g.nx * g.ny * g.nz
        self.keep = []
        self.grid = A.KwGrid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.dt, g.cfl,
                             (C.c_int32 * 3)(*g.pml_size), (C.c_double * 3)(*g.pml_alpha))
        fields = {}
        for name in ("c0", "rho0", "alpha0", "bona"):
            arr, sc_val = _map_or_scalar(getattr(m, name), n)
            self.keep.append(arr)
            fields[name] = (_fptr(arr), sc_val)
        flags = (A.KW_NONLINEAR if m.nonlinear else 0) | (A.KW_ABSORBING if m.absorbing else 0)
        self.medium = A.KwMedium(fields["c0"][0], fields["c0"][1], fields["rho0"][0],
                                 fields["rho0"][1], fields["alpha0"][0], fields["alpha0"][1],
                                 fields["bona"][0], fields["bona"][1], m.alpha_power, m.c_ref,
                                 flags)
        s = sc.source
        if s is not None and len(s.index) > 0:
            idx = np.ascontiguousarray(s.index, np.int64)
            elem = None if s.element is None else np.ascontiguousarray(s.element, np.int32)
            amp = np.ascontiguousarray(s.amp, np.float32)
            ph = np.ascontiguousarray(s.phase, np.float32)
            sig = None if s.signal is None else np.ascontiguousarray(s.signal, np.float32)
            self.keep += [idx, elem, amp, ph, sig]
            self.source = A.KwSource(idx.size, idx.ctypes.data_as(_P(C.c_int64)),
                                     None if elem is None else elem.ctypes.data_as(_P(C.c_int32)),
                                     amp.size, _fptr(amp), _fptr(ph), s.freq, _fptr(sig),
                                     0 if sig is None else sig.shape[1], int(s.kind), int(s.axis))
        else:
            self.source = A.KwSource()
        z = sc.sensor
        if z.index is not None:
            sidx = np.ascontiguousarray(z.index, np.int64)
            self.keep.append(sidx)
            self.sensor = A.KwSensor(z.record, sidx.size, sidx.ctypes.data_as(_P(C.c_int64)),
                                     z.record_start, z.series_capacity, z.n_harmonics,
                                     z.harmonic_freq)
        else:
            self.sensor = A.KwSensor(z.record, 0, None, z.record_start, z.series_capacity,
                                     z.n_harmonics, z.harmonic_freq)

    def args(self):
        return (C.byref(self.grid), C.byref(self.medium), C.byref(self.source),
                C.byref(self.sensor))


def workspace_size(sc: Scenario) -> int:
    lib = A.load()
    m = _Marshalled(sc)
    n = lib.kw_workspace_size(*m.args())
    if n == 0:
        raise A.KwError(A.KW_EINVAL, lib.kw_last_error().decode())
    return int(n)


class Prepared:
    """Host part of a simulation's set-up (kw_prepare): validation, FFT plans,
    float64 operator tables and medium maps.  It makes no device call, so it
    may be built in any thread; Simulation(..., prepared=p) then only uploads."""

    def __init__(self, sc: Scenario):
        self.lib = A.load()
        self.scenario = sc
        m = _Marshalled(sc)
        handle = C.c_void_p()
        A.check(self.lib.kw_prepare(*m.args(), C.byref(handle)))
        self.handle = handle
        self.workspace_bytes = int(self.lib.kw_plan_workspace_size(handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.kw_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _hip_runtime():
    """The HIP runtime already in the process (torch's, which libkw.so binds
    to as well): a stream of our own is created there."""
    global _hip
    if _hip is None:
        A.load()
        lib = C.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
        lib.hipStreamCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        lib.hipStreamCreateWithFlags.restype = C.c_int
        lib.hipStreamDestroy.argtypes = [C.c_void_p]
        lib.hipStreamDestroy.restype = C.c_int
        _hip = lib
    return _hip


_HIP_STREAM_NON_BLOCKING = 1


def _own_stream(device: torch.device):
    """A new non-blocking HIP stream at the default priority (torch.cuda.Stream
    hands out one of 32 pooled streams per device in turn, so simulations that
    live long enough would end up sharing one)."""
    hip = _hip_runtime()
    handle = C.c_void_p()
    with torch.cuda.device(device):
        rc = hip.hipStreamCreateWithFlags(C.byref(handle), _HIP_STREAM_NON_BLOCKING)
    if rc != 0:
        raise A.KwError(A.KW_EDEVICE, "hipStreamCreateWithFlags failed (%d)" % rc)
    return handle.value, torch.cuda.ExternalStream(handle.value, device=device)


def static_workspace_size(sc: Scenario) -> int:
    """Workspace bytes of a simulation whose six spectral scratch arrays live in
    the library's static array (kw_create_static)."""
    g = sc.grid
    spectrum = 256 * ((4 * g.nx * g.ny * g.nz + 255) // 256)
    return workspace_size(sc) - 6 * spectrum


class Simulation:
    """One simulation on the GPU.  It runs on a HIP stream of its own (or on
    `stream` when one is given); the device workspace is a torch tensor.  With
    static_scratch the spectral scratch arrays come from the library's static
    array (kw_create_static): a smaller workspace, and simulations made so on
    one GPU must not run at the same time."""

    def __init__(self, sc: Scenario, device: str = "cuda", stream: Optional[torch.cuda.Stream] = None,
                 graph_steps: Optional[int] = None, tune: bool = True,
                 prepared: Optional[Prepared] = None, static_scratch: bool = False):
        self.lib = A.load()
        self.scenario = sc
        self.device = torch.device(device)
        self.handle = None
        self._own = None
        if static_scratch and prepared is not None:
            raise ValueError("static_scratch builds its own set-up (no prepared plan)")
        own_prep = prepared is None and not static_scratch
        prep = Prepared(sc) if own_prep else prepared
        try:
            nbytes = static_workspace_size(sc) if static_scratch else prep.workspace_bytes
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            if stream is None:
                self._own, self.stream = _own_stream(self.device)
            else:
                self.stream = stream
            # the workspace is allocated on the current stream: order it before the
            # simulation's stream.  No record_stream: close() synchronises the
            # simulation's stream before the workspace is released
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            handle = C.c_void_p()
            if static_scratch:
                m = _Marshalled(sc)
                A.check(self.lib.kw_create_static(*m.args(), C.c_void_p(self.workspace.data_ptr()),
                                                  C.c_size_t(nbytes),
                                                  C.c_void_p(self.stream.cuda_stream),
                                                  C.byref(handle)))
            else:
                A.check(self.lib.kw_create_prepared(prep.handle,
                                                    C.c_void_p(self.workspace.data_ptr()),
                                                    C.c_size_t(nbytes),
                                                    C.c_void_p(self.stream.cuda_stream),
                                                    C.byref(handle)))
            self.handle = handle
        except Exception:
            self.close()
            raise
        finally:
            if own_prep:
                prep.close()
        self.npts = sc.grid.npts
        if graph_steps is not None:
            A.check(self.lib.kw_set_graph(self.handle, int(graph_steps)))
        self.plans = {}
        if tune:
            # schedules chosen by the autotuner for these transform lengths, if cached
            from .autotune import lookup
            for axis, (rad, tile) in lookup(sc.grid).items():
                try:
                    self.set_plan(axis, rad, tile)
                    self.plans[axis] = (rad, tile)
                except A.KwError:
                    pass

    # ------------------------------------------------------------------
    def step(self, n: int = 1):
        A.check(self.lib.kw_step(self.handle, int(n)))

    def gather(self, what: int, device: bool = True):
        nb = self.lib.kw_gather_bytes(self.handle, what)
        if nb < 0:
            raise A.KwError(A.KW_EINVAL, "unknown gather target")
        n = max(nb // 4, 1)
        if device:
            out = torch.empty(n, dtype=torch.float32, device=self.device)
            ptr, isdev = out.data_ptr(), 1
        else:
            out = np.empty(n, np.float32)
            ptr, isdev = out.ctypes.data, 0
        A.check(self.lib.kw_gather(self.handle, what, C.c_void_p(ptr), C.c_size_t(n * 4), isdev))
        return out[: nb // 4]

    def set_field(self, field: int, values):
        if isinstance(values, torch.Tensor):
            v = values.detach().to(self.device, torch.float32).contiguous().reshape(-1)
            torch.cuda.current_stream(self.device).synchronize()
            A.check(self.lib.kw_set_field(self.handle, field, C.c_void_p(v.data_ptr()), 1))
        else:
            v = np.ascontiguousarray(np.asarray(values, np.float32).reshape(-1))
            if v.size != self.npts:
                raise ValueError("field has %d values, grid has %d" % (v.size, self.npts))
            A.check(self.lib.kw_set_field(self.handle, field, C.c_void_p(v.ctypes.data), 0))

    def get_field(self, field: int) -> np.ndarray:
        out = np.empty(self.npts, np.float32)
        A.check(self.lib.kw_gather_field(self.handle, field, C.c_void_p(out.ctypes.data), 0))
        return out

    def state_bytes(self) -> int:
        return int(self.lib.kw_state_bytes(self.handle))

    def save(self, device: bool = True):
        """Snapshot of the evolving state (uint8 tensor on the GPU, or a numpy
        array in host memory when device is False)."""
        nb = self.state_bytes()
        if device:
            out = torch.empty(nb, dtype=torch.uint8, device=self.device)
            ptr, isdev = out.data_ptr(), 1
            torch.cuda.current_stream(self.device).synchronize()
        else:
            out = np.empty(nb, np.uint8)
            ptr, isdev = out.ctypes.data, 0
        A.check(self.lib.kw_save(self.handle, C.c_void_p(ptr), C.c_size_t(nb), isdev))
        return out

    def load(self, snapshot):
        """Restore a snapshot taken with save() from a simulation of the same set-up."""
        if isinstance(snapshot, torch.Tensor):
            v = snapshot.contiguous()
            if v.is_cuda:
                torch.cuda.current_stream(v.device).synchronize()
                A.check(self.lib.kw_load(self.handle, C.c_void_p(v.data_ptr()),
                                         C.c_size_t(v.numel() * v.element_size()), 1))
                return
            snapshot = v.numpy()
        a = np.ascontiguousarray(snapshot, np.uint8)
        A.check(self.lib.kw_load(self.handle, C.c_void_p(a.ctypes.data), C.c_size_t(a.size), 0))

    def profile(self, on: bool):
        A.check(self.lib.kw_profile(self.handle, 1 if on else 0))

    def set_plan(self, axis: int, radices, tile: int = 0):
        arr = (C.c_int32 * len(radices))(*radices) if radices else None
        A.check(self.lib.kw_set_plan(self.handle, axis, arr, len(radices) if radices else 0, tile))

    def stats(self) -> dict:
        st = A.KwStats()
        A.check(self.lib.kw_stats(self.handle, C.byref(st)))
        classes = {}
        for i in range(st.n_classes):
            name = st.class_name[i].value.decode()
            classes[name] = dict(ms=st.class_ms[i], launches=st.class_launches[i],
                                 bytes=st.class_bytes[i])
        return dict(steps=st.steps, nonfinite_step=st.nonfinite_step, dt=st.dt, c_ref=st.c_ref,
                    workspace_bytes=st.workspace_bytes,
                    fft_forward_per_step=st.fft_forward_per_step,
                    fft_inverse_per_step=st.fft_inverse_per_step,
                    kernels_per_step=st.kernels_per_step, classes=classes)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        """Wait for the simulation's work, free its host state, release the
        workspace and destroy the stream it owns (in that order: the workspace
        goes back to torch only once nothing on the stream can touch it)."""
        if getattr(self, "handle", None):
            self.stream.synchronize()
            self.lib.kw_destroy(self.handle)
            self.handle = None
        self.workspace = None
        if getattr(self, "_own", None):
            self.stream.synchronize()
            _hip_runtime().hipStreamDestroy(C.c_void_p(self._own))
            self._own = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
