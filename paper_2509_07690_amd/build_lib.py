"""Build libhylu.so (host analysis + gfx950 kernels + C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhylu.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are disabled in every device compile
DEV_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build(force: bool = True, jobs: int = 4) -> str:
    if not force and os.path.exists(OUT):
        return OUT
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src, kind in (("host_order.cpp", "host"), ("host_symbolic.cpp", "host"),
                      ("hylu_api.cpp", "hip"), ("kernels.hip", "hip"), ("symbolic.hip", "hip")):
        obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        path = os.path.join(CSRC, src)
        if kind == "host":
            cmd = ["g++"] + HOST_FLAGS + ["-c", path, "-o", obj]
        else:
            cmd = [HIPCC] + DEV_FLAGS + ["-x", "hip", "-c", path, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
    if failed:
        raise RuntimeError("build failed")
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
