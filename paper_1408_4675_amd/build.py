"""Build the HIP library libkw.so in-tree for gfx950 (hipcc, no JIT cache).

Usage: python -m paper_1408_4675_amd.build  (or call build()).
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkw.so")
ARCH = os.environ.get("KW_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r.stdout


HIP_SOURCES = ("kernels_yz.hip", "kernels_x.hip", "kernels_util.hip", "kernels_adj.hip",
               "static_scratch.hip")
PROBE_SOURCES = ("zcol_copy.hip",)


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every HIP translation unit for gfx950 (in parallel) and link
    libkw.so next to this file."""
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="kwbuild_") as tmp:
        jobs = []
        objs = []
        for src in HIP_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            cmd = ([hipcc, "-x", "hip", "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS
                   + list(extra_flags) + ["-c", os.path.join(CSRC, src), "-o", obj])
            jobs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                               stderr=subprocess.STDOUT, text=True)))
        # the measurement probes are programs of their own (built and run by
        # profiling.py); compiled here too so that a build checks them
        for src in PROBE_SOURCES:
            cmd = ([hipcc, "-x", "hip", "--offload-arch=" + ARCH, "-O3", "-std=c++17"] + DEVICE_FLAGS
                   + ["-c", os.path.join(HERE, "probes", src), "-o", os.path.join(tmp, src + ".o")])
            jobs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                               stderr=subprocess.STDOUT, text=True)))
        e_obj = os.path.join(tmp, "engine.o")
        objs.append(e_obj)
        out = _run([hipcc] + COMMON + ["-c", os.path.join(CSRC, "engine.cpp"), "-o", e_obj])
        for cmd, pr in jobs:
            o, _ = pr.communicate()
            out += o
            if pr.returncode != 0:
                sys.stderr.write(o)
                raise RuntimeError("command failed: " + " ".join(cmd))
        tmp_lib = LIB + ".tmp"
        out += _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp_lib])
        os.replace(tmp_lib, LIB)
    if verbose and out.strip():
        print(out)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
