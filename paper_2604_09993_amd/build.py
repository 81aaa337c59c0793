"""Build the gfx950 shared library ``libcis.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcis.so")
SOURCES = ["cis.hip", "cis_adjoint.hip", "cis_batch.hip", "cis_blocked.hip", "cis_split.hip",
           "cis_impact.hip", "cis_rkf.hip", "cis_paper.hip", "cis_debug.hip",
           "cis_host.cpp", "cis_ldl.cpp"]
HEADERS = ["cis_model.hpp", "cis_body.hpp", "cis_host.hpp", "cis_launch.hpp", "cis_split.hpp",
           "cis_debug.hpp",
           os.path.join("..", "..", "include", "cis.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++20", f"--offload-arch={ARCH}", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _objects(build_dir):
    return [os.path.join(build_dir, os.path.splitext(s)[0] + ".o") for s in SOURCES]


def build(verbose: bool = False, jobs: int = 3) -> str:
    """Compile every source (in parallel) and link libcis.so; always rebuilds."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src, obj in zip(SOURCES, _objects(build_dir)):
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
        elif verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + _objects(build_dir)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    files = [os.path.join(CSRC, f) for f in SOURCES + HEADERS]
    return any(os.path.getmtime(f) > t for f in files if os.path.exists(f))


if __name__ == "__main__":
    print(build(verbose=True))
