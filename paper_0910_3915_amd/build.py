"""Build libscdrop.so (HIP, gfx950) in-tree with hipcc.

Each source is compiled to its own object in parallel (the kernels of one
file call no device code of another), then the objects are linked into the
shared library.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libscdrop.so")
SOURCES = ["step.hip", "observe.hip", "adjoint.hip", "api.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="scdrop_build_") as tmp:
        objs, procs = [], []
        for s in SOURCES:
            o = os.path.join(tmp, os.path.splitext(s)[0] + ".o")
            cmd = [hipcc] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", o]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd)))
            objs.append(o)
        failed = [s for s, p in procs if p.wait() != 0]
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(failed))
        # roctx: the entry points' trace ranges (rocprofv3 --marker-trace)
        cmd = ([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs +
               ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-o", LIB + ".tmp"])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
