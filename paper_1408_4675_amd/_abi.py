"""ctypes mirror of include/kw.h.  Argument marshalling only: every step of
the solver runs in the HIP library libkw.so; this module never computes."""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkw.so")

KW_OK = 0
KW_EINVAL = -1
KW_EUNSUPPORTED = -2
KW_ENOMEM = -3
KW_EDEVICE = -4
KW_ESTATE = -5
KW_ENONFINITE = -6
STATUS_NAMES = {0: "KW_OK", -1: "KW_EINVAL", -2: "KW_EUNSUPPORTED", -3: "KW_ENOMEM",
                -4: "KW_EDEVICE", -5: "KW_ESTATE", -6: "KW_ENONFINITE"}

KW_SOURCE_MASS = 0
KW_SOURCE_FORCE = 1
KW_SOURCE_PRESSURE = 2

KW_NONLINEAR = 1
KW_ABSORBING = 2

KW_REC_P_MAX = 1
KW_REC_P_RMS = 2
KW_REC_P_SERIES = 4
KW_REC_P_FINAL = 8
KW_REC_U_FINAL = 16
KW_REC_INTENSITY = 32
KW_REC_P_MIN = 64
KW_REC_HARMONICS = 128
KW_REC_U_SERIES = 256

KW_FIELD_P = 1
KW_FIELD_UX = 2
KW_FIELD_UY = 3
KW_FIELD_UZ = 4
KW_FIELD_RHOX = 5
KW_FIELD_RHOY = 6
KW_FIELD_RHOZ = 7

# every symbol include/kw.h declares
EXPORTS = ("kw_workspace_size", "kw_create", "kw_prepare", "kw_plan_workspace_size",
           "kw_create_prepared", "kw_plan_destroy", "kw_create_static", "kw_step", "kw_gather", "kw_gather_bytes",
           "kw_set_field", "kw_gather_field", "kw_profile", "kw_stats", "kw_set_graph",
           "kw_set_plan", "kw_state_bytes", "kw_save", "kw_load", "kw_adjoint_workspace_size",
           "kw_adjoint_create", "kw_adjoint_objective", "kw_adjoint_step", "kw_adjoint_source_gradient",
           "kw_adjoint_record_bytes", "kw_adjoint_record", "kw_adjoint_step_record",
           "kw_adjoint_gradient", "kw_adjoint_destroy", "kw_destroy", "kw_last_error")


class KwGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double), ("cfl", C.c_double),
                ("pml_size", C.c_int32 * 3), ("pml_alpha", C.c_double * 3)]


class KwMedium(C.Structure):
    _fields_ = [("c0", C.POINTER(C.c_float)), ("c0_scalar", C.c_double),
                ("rho0", C.POINTER(C.c_float)), ("rho0_scalar", C.c_double),
                ("alpha0", C.POINTER(C.c_float)), ("alpha0_scalar", C.c_double),
                ("bona", C.POINTER(C.c_float)), ("bona_scalar", C.c_double),
                ("alpha_power", C.c_double), ("c_ref", C.c_double), ("flags", C.c_uint32)]


class KwSource(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("index", C.POINTER(C.c_int64)),
                ("element", C.POINTER(C.c_int32)), ("n_elements", C.c_int32),
                ("amp", C.POINTER(C.c_float)), ("phase", C.POINTER(C.c_float)),
                ("freq", C.c_double), ("signal", C.POINTER(C.c_float)),
                ("n_samples", C.c_int32), ("kind", C.c_int32), ("axis", C.c_int32)]


class KwSensor(C.Structure):
    _fields_ = [("record", C.c_uint32), ("n_points", C.c_int64),
                ("index", C.POINTER(C.c_int64)), ("record_start", C.c_int32),
                ("series_capacity", C.c_int32), ("n_harmonics", C.c_int32),
                ("harmonic_freq", C.c_double)]


class KwStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("nonfinite_step", C.c_int64), ("dt", C.c_double),
                ("c_ref", C.c_double), ("workspace_bytes", C.c_int64),
                ("fft_forward_per_step", C.c_int32), ("fft_inverse_per_step", C.c_int32),
                ("kernels_per_step", C.c_int32), ("n_classes", C.c_int32),
                ("class_name", (C.c_char * 24) * 16), ("class_ms", C.c_double * 16),
                ("class_launches", C.c_int64 * 16), ("class_bytes", C.c_double * 16)]


class KwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


_lib = None
_lock = threading.Lock()


def load(path: str = LIB_PATH):
    """Load libkw.so (raise if it has not been built)."""
    with _lock:
        return _load(path)


def _load(path):
    global _lib
    if _lib is not None:
        return _lib
    # torch first: it brings the HIP runtime the workspace tensors live in, and
    # libkw.so must bind to that same runtime rather than load a second one
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise FileNotFoundError("HIP library %s is missing: run paper_1408_4675_amd.build "
                                "(or __graft_entry__.build()) first" % path)
    lib = C.CDLL(path)
    P = C.POINTER
    lib.kw_workspace_size.restype = C.c_size_t
    lib.kw_workspace_size.argtypes = [P(KwGrid), P(KwMedium), P(KwSource), P(KwSensor)]
    lib.kw_create.restype = C.c_int
    lib.kw_create.argtypes = [P(KwGrid), P(KwMedium), P(KwSource), P(KwSensor), C.c_void_p,
                              C.c_size_t, C.c_void_p, P(C.c_void_p)]
    lib.kw_prepare.restype = C.c_int
    lib.kw_prepare.argtypes = [P(KwGrid), P(KwMedium), P(KwSource), P(KwSensor), P(C.c_void_p)]
    lib.kw_plan_workspace_size.restype = C.c_size_t
    lib.kw_plan_workspace_size.argtypes = [C.c_void_p]
    lib.kw_create_prepared.restype = C.c_int
    lib.kw_create_prepared.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                       P(C.c_void_p)]
    lib.kw_create_static.restype = C.c_int
    lib.kw_create_static.argtypes = [P(KwGrid), P(KwMedium), P(KwSource), P(KwSensor), C.c_void_p,
                                     C.c_size_t, C.c_void_p, P(C.c_void_p)]
    lib.kw_plan_destroy.restype = C.c_int
    lib.kw_plan_destroy.argtypes = [C.c_void_p]
    lib.kw_step.restype = C.c_int
    lib.kw_step.argtypes = [C.c_void_p, C.c_int32]
    lib.kw_gather.restype = C.c_int
    lib.kw_gather.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_size_t, C.c_int]
    lib.kw_gather_bytes.restype = C.c_int64
    lib.kw_gather_bytes.argtypes = [C.c_void_p, C.c_uint32]
    lib.kw_set_field.restype = C.c_int
    lib.kw_set_field.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
    lib.kw_gather_field.restype = C.c_int
    lib.kw_gather_field.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int]
    lib.kw_profile.restype = C.c_int
    lib.kw_profile.argtypes = [C.c_void_p, C.c_int]
    lib.kw_stats.restype = C.c_int
    lib.kw_stats.argtypes = [C.c_void_p, P(KwStats)]
    lib.kw_set_graph.restype = C.c_int
    lib.kw_set_graph.argtypes = [C.c_void_p, C.c_int32]
    lib.kw_set_plan.restype = C.c_int
    lib.kw_set_plan.argtypes = [C.c_void_p, C.c_int, P(C.c_int32), C.c_int32, C.c_int32]
    lib.kw_state_bytes.restype = C.c_int64
    lib.kw_state_bytes.argtypes = [C.c_void_p]
    lib.kw_save.restype = C.c_int
    lib.kw_save.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    lib.kw_load.restype = C.c_int
    lib.kw_load.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    lib.kw_adjoint_workspace_size.restype = C.c_size_t
    lib.kw_adjoint_workspace_size.argtypes = [C.c_void_p, C.c_int32]
    lib.kw_adjoint_create.restype = C.c_int
    lib.kw_adjoint_create.argtypes = [C.c_void_p, P(C.c_float), C.c_int32, C.c_void_p,
                                      C.c_size_t, P(C.c_void_p)]
    lib.kw_adjoint_objective.restype = C.c_int
    lib.kw_adjoint_objective.argtypes = [C.c_void_p, P(C.c_double)]
    lib.kw_adjoint_step.restype = C.c_int
    lib.kw_adjoint_step.argtypes = [C.c_void_p, C.c_int32]
    lib.kw_adjoint_record_bytes.restype = C.c_int64
    lib.kw_adjoint_record_bytes.argtypes = [C.c_void_p]
    lib.kw_adjoint_record.restype = C.c_int
    lib.kw_adjoint_record.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    lib.kw_adjoint_step_record.restype = C.c_int
    lib.kw_adjoint_step_record.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]
    lib.kw_adjoint_source_gradient.restype = C.c_int
    lib.kw_adjoint_source_gradient.argtypes = [C.c_void_p, P(C.c_double), C.c_size_t]
    lib.kw_adjoint_gradient.restype = C.c_int
    lib.kw_adjoint_gradient.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.kw_adjoint_destroy.restype = C.c_int
    lib.kw_adjoint_destroy.argtypes = [C.c_void_p]
    lib.kw_destroy.restype = C.c_int
    lib.kw_destroy.argtypes = [C.c_void_p]
    lib.kw_last_error.restype = C.c_char_p
    lib.kw_last_error.argtypes = []
    _lib = lib
    return lib


def check(code: int):
    if code != KW_OK:
        raise KwError(code, load().kw_last_error().decode(errors="replace"))
    return code
