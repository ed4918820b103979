"""The engine's host code (set-up, error paths) on the CPU under
AddressSanitizer and ThreadSanitizer.

engine.cpp is built with g++ against a host stand-in of the HIP runtime and
of the kernel launchers (tests/native/hip_host_stub.cpp: "device memory" is
host memory, copies are memcpy, fills write their values).  The driver
(tests/native/engine_host_test.cpp) checks that kw_prepare,
kw_create_prepared and kw_create running in 8 threads at once leave exactly
the workspace bytes of a serial run, that failing device calls return
their status unchanged (kw_gather_field of the pressure included), and that
kw_set_plan accepts a schedule for every kind of FFT engine instantiation and
refuses schedules that do not factor the length."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1408_4675_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
HIP_INCLUDE = "/opt/rocm/include"


@pytest.mark.parametrize("sanitizer", ["address", "thread"])
def test_engine_host_code_under_sanitizer(sanitizer, tmp_path):
    if shutil.which("g++") is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip")):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / ("engine_host_" + sanitizer))
    build = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-D__HIP_PLATFORM_AMD__",
             "-I", HIP_INCLUDE, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-fsanitize=" + sanitizer, os.path.join(CSRC, "engine.cpp"),
             os.path.join(NATIVE, "hip_host_stub.cpp"), os.path.join(NATIVE, "engine_host_test.cpp"),
             "-o", exe]
    r = subprocess.run(build, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    for mode in ("threads", "errors", "plans"):
        r = subprocess.run([exe, mode], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                           timeout=600, env=env)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "Sanitizer" not in r.stderr, r.stderr
