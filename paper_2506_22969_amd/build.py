"""Build libsparstencil.so for gfx950 in-tree with hipcc.

The host planner is compiled without floating-point contraction so that its
tables are reproducible; all HIP code gets -packed-fp32-ops disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsparstencil.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-Wall", "-Wno-unused-variable", "-Wno-unused-result"]
SOURCES = ["mma2d_f32_r3.hip", "mma2d_f32_r1.hip", "mma2d_f32_r2.hip", "mma2d_f16.hip", "mma2d_planes.hip",
           "mma2d_planes3.hip", "mma3d.hip",
           "mma2d_f64.hip", "mma1d.hip", "direct2d.hip", "mma2d.hip", "direct.hip", "runtime.hip", "server.hip", "probe.hip"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(jobs: int = 6) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    cmds = []
    # planner: host-only C++, exact rounding order
    obj = os.path.join(out_dir, "planner.o")
    cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-c",
                 os.path.join(CSRC, "planner.cpp"), "-o", obj])
    objs.append(obj)
    for src in SOURCES:
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        cmds.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    procs = []
    for c in cmds:
        procs.append((c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for pc in procs:
        _wait(pc)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def _wait(pc):
    cmd, proc = pc
    out, _ = proc.communicate()
    if proc.returncode != 0:
        sys.stderr.write(out)
        raise RuntimeError("command failed: " + " ".join(cmd))
    if out and "warning" in out and "packed-fp32-ops" not in out:
        sys.stderr.write(out)


if __name__ == "__main__":
    print(build())
