"""C ABI checks that need no GPU: the library loads, exports every function
include/kw.h declares, and validates its inputs before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1408_4675_amd import _abi as A
from paper_1408_4675_amd import scenarios as sc
from paper_1408_4675_amd.simulation import _Marshalled

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.fail("libkw.so is not built (run __graft_entry__.build())")
    return A.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "kw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kw_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(A.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def _ws(lib, scen):
    m = _Marshalled(scen)
    return lib.kw_workspace_size(*m.args())


def test_workspace_size_accounts_for_every_array(lib):
    scen = sc.small_case(48, 20, 18, seed=0)
    n = scen.grid.npts
    ws = _ws(lib, scen)
    # 3 u + 3 rho + rho_total + 7 spectra + 8 medium maps + p_max + p_sum2 fields
    assert ws >= (7 + 7 + 8 + 2) * 4 * n
    assert ws < (7 + 7 + 8 + 2) * 4 * n + 4 * 1024 * 1024


def test_workspace_of_large_homogeneous_grid_fits_one_gpu(lib):
    scen = sc.Scenario("big", sc.Grid(1024, 1024, 1024, 5e-5, 5e-5, 5e-5, dt=1e-8),
                       sc.Medium(**sc.WATER), None,
                       sc.Sensor(record=sc.REC_P_SERIES, index=np.array([5], np.int64),
                                 series_capacity=100), 0)
    ws = _ws(lib, scen)
    field = 1024 ** 3 * 4
    assert 14 * field <= ws < 14 * field + (64 << 20)     # 6 state + rho + 7 spectra
    assert ws < 288e9


def test_table1_memory_per_matrix():
    # Table 1: one FP32 matrix of 667^3 points is 1.1 GB and of 1333^3 is 8.8 GB
    for n, gb in ((667, 1.1), (1333, 8.8)):
        assert abs(n ** 3 * 4 / 2 ** 30 - gb) < 0.1


BAD = [
    ("odd nx", dict(nx=33)),
    ("7 factor", dict(ny=28)),
    ("too small", dict(nz=2)),
    ("pml too big", dict(pml=20)),
    ("y = 1", dict(y=1.0)),
    ("negative dx", dict(dx=-1.0)),
    ("unsorted source", dict(unsorted=True)),
    ("source out of grid", dict(src_oob=True)),
    ("series without index", dict(series_all=True)),
    ("velocity series without index", dict(useries_all=True)),
    ("unknown source kind", dict(kind=7)),
    ("force axis out of range", dict(kind=1, axis=3)),
    ("too many harmonics", dict(harmonics=17)),
    ("harmonics without frequency", dict(harmonics=2, no_source=True)),
    ("unknown record bit", dict(record=1 << 12)),
    ("record_start 0", dict(record_start=0)),
]


@pytest.mark.parametrize("name,kw", BAD, ids=[b[0] for b in BAD])
def test_validation_rejects_bad_inputs(lib, name, kw):
    nx, ny, nz = kw.get("nx", 32), kw.get("ny", 20), kw.get("nz", 18)
    scen = sc.small_case(32, 20, 18, seed=1)
    g = scen.grid
    g.nx, g.ny, g.nz = nx, ny, nz
    if "pml" in kw:
        g.pml_size = (kw["pml"],) * 3
    if "dx" in kw:
        g.dx = kw["dx"]
    scen.medium = sc.Medium(**sc.WATER, alpha_power=kw.get("y", 1.5))
    if kw.get("unsorted"):
        scen.source.index = scen.source.index[::-1].copy()
    if kw.get("src_oob"):
        scen.source.index = np.array([0, 10 ** 9], np.int64)
    if kw.get("series_all"):
        scen.sensor = sc.Sensor(record=sc.REC_P_SERIES, index=None, series_capacity=4)
    if kw.get("useries_all"):
        scen.sensor = sc.Sensor(record=sc.REC_U_SERIES, index=None, series_capacity=4)
    if "kind" in kw:
        scen.source.kind = kw["kind"]
        scen.source.axis = kw.get("axis", 0)
    if "harmonics" in kw:
        scen.sensor = sc.Sensor(record=sc.REC_HARMONICS, n_harmonics=kw["harmonics"])
    if kw.get("no_source"):
        scen.source = None
    if "record" in kw:
        scen.sensor = sc.Sensor(record=kw["record"])
    if "record_start" in kw:
        scen.sensor = sc.Sensor(record=sc.REC_P_MAX, record_start=kw["record_start"])
    assert _ws(lib, scen) == 0
    assert lib.kw_last_error().decode()
    m = _Marshalled(scen)
    out = C.c_void_p()
    rc = lib.kw_create(*m.args(), C.c_void_p(256), C.c_size_t(1 << 40), None, C.byref(out))
    assert rc in (A.KW_EINVAL, A.KW_EUNSUPPORTED)
    assert not out.value


def test_create_rejects_small_workspace_before_device_use(lib):
    scen = sc.small_case(32, 20, 18, seed=1)
    m = _Marshalled(scen)
    need = lib.kw_workspace_size(*m.args())
    out = C.c_void_p()
    rc = lib.kw_create(*m.args(), C.c_void_p(256), C.c_size_t(need - 1), None, C.byref(out))
    assert rc == A.KW_ENOMEM


def test_null_safety(lib):
    assert lib.kw_destroy(None) == A.KW_OK
    assert lib.kw_step(None, 1) == A.KW_EINVAL
    assert lib.kw_gather(None, 1, None, 0, 0) == A.KW_EINVAL
