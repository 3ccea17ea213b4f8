"""Builds libwavetile.so in-tree (host C++ with g++, device code with hipcc
for gfx950), then links it against the HIP runtime and hipRTC.

Usage: python paper_1909_07190_amd/build.py   (or __graft_entry__.build())
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libwavetile.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["ir.cpp", "geometry.cpp", "codegen.cpp", "sched.cpp", "fusion.cpp",
                "cost.cpp", "prof.cpp", "autotune.cpp", "batch.cpp", "mlp.cpp", "train_db.cpp", "jit.cpp", "runtime.cpp",
                "capi.cpp"]
DEVICE_SOURCES: list[str] = ["mlp.hip", "copyref.hip", "scratch.hip", "histzero.hip"]
# Packed-FP32 VALU forms are disabled in every HIP compilation.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
              "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]


def _embed_device_header():
    src = open(os.path.join(CSRC, "device", "wt_device.h")).read()
    if ")WTDEV\"" in src:
        raise RuntimeError("device header contains the raw-string delimiter")
    text = ("// Generated from device/wt_device.h by build.py; do not edit.\n"
            "static const char kWtDeviceSrc[] = R\"WTDEV(" + src + ")WTDEV\";\n")
    path = os.path.join(CSRC, "wt_device_src.inc")
    if not os.path.exists(path) or open(path).read() != text:
        with open(path, "w") as f:
            f.write(text)


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compiles every source (always, even when a library exists) and links."""
    os.makedirs(BUILD, exist_ok=True)
    _embed_device_header()
    jobs = []
    for s in HOST_SOURCES:
        if not os.path.exists(os.path.join(CSRC, s)):
            continue
        obj = os.path.join(BUILD, s + ".o")
        jobs.append((["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", obj], obj))
    for s in DEVICE_SOURCES:
        obj = os.path.join(BUILD, s + ".o")
        jobs.append(([f"{ROCM}/bin/hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", obj], obj))
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        outs = list(ex.map(lambda j: _run(j[0]), jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [o for _, o in jobs]
    tmp = OUT + ".tmp"
    link = [f"{ROCM}/bin/hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp,
            f"-L{ROCM}/lib", "-lamdhip64", "-lhiprtc", f"-Wl,-rpath,{ROCM}/lib"]
    _run(link)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
