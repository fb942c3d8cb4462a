"""Build steps for the native parts of the package (run on any host; no GPU needed).

* ``libtriadgen.so``  - seeded input generators (g++ / OpenMP)
* ``libtriad.so``     - the census C-ABI and its HIP kernels for gfx950 (hipcc)
"""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_SOURCES = ["census.hip", "costmodel.hip", "csr_build.hip", "update.hip", "profile.hip", "host.cpp"]


def gen_lib_path():
    return os.path.join(PKG, "libtriadgen.so")


def triad_lib_path():
    return os.path.join(PKG, "libtriad.so")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build_gen():
    out = gen_lib_path()
    tmp = out + ".tmp"
    _run(["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
          os.path.join(PKG, "gen", "graphgen.cpp"), "-o", tmp])
    os.replace(tmp, out)
    return out


def hip_flags():
    return [
        "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
        # keep the compiler from forming packed-FP32 VALU ops
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    ]


def build_triad():
    out = triad_lib_path()
    tmp = out + ".tmp"
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    _run([HIPCC, *hip_flags(), "-shared", *srcs, "-o", tmp, "-lpthread"])
    os.replace(tmp, out)
    return out


def build_all():
    build_gen()
    build_triad()
