"""Builds the xg C-ABI library (libxg.so) in-tree with hipcc.

The library is host code (planner, emitter, hiprtc driver, launches) plus one
device array (the workspace of the no-allocation adjoint entry point); the
kernels it runs are generated per program and compiled for gfx950 at run
time by hiprtc.  Run: python -m paper_2408_09662_amd.build
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxg.so")
# compile helper: the library runs several of these at once to compile the
# chunks of a large program in parallel
RTC = os.path.join(HERE, "xg-rtc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["xg_ir.cpp", "xg_plan.cpp", "xg_emit.cpp", "xg_adjoint.cpp", "xg_jit.cpp",
           "xg_api.cpp", "xg_batch.cpp", "xg_static.hip"]


def build(verbose: bool = False) -> str:
    objs = []
    common = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"),
              "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for s in SOURCES:
        src = os.path.join(SRC, s)
        obj = os.path.join(bdir, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC, *common, "-c", src, "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    rtc_cmd = [HIPCC, "-O2", "-std=c++17", "-Wall", os.path.join(SRC, "xg_rtc_main.cpp"),
               "-o", RTC + ".tmp", "-lhiprtc"]
    procs.append((rtc_cmd, subprocess.Popen(rtc_cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 target feature
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed = True
            sys.stderr.write(" ".join(cmd) + "\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("building libxg.so failed")
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc", "-lpthread"],
                   check=True)
    os.replace(tmp, LIB)
    os.replace(RTC + ".tmp", RTC)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
