"""Build libvuda.so (HIP kernels + C-ABI runtime) for gfx950, in-tree."""
import glob
import hashlib
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libvuda.so")

MANIFEST = os.path.join(LIBDIR, "libvuda.sources.json")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # bit-exact agreement with the CPU oracle: no contraction into FMA,
    # correctly rounded fp32 division and square root (the HIP default)
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def source_files():
    """Every file the library is compiled from: the HIP sources, their headers
    and the C-ABI header."""
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")) +
                  glob.glob(os.path.join(ROOT, "include", "*.h")))


def source_digests():
    """{path relative to the repository root: sha256 of its bytes}."""
    out = {}
    for f in source_files():
        with open(f, "rb") as fh:
            out[os.path.relpath(f, ROOT)] = hashlib.sha256(fh.read()).hexdigest()
    return out


def build(verbose: bool = False, jobs: int = 4) -> str:
    digests = source_digests()  # taken before compiling: what the objects are built from
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objdir = os.path.join(LIBDIR, "_obj")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for s in srcs:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], "-c", *inc, s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            s0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s0}")
    for s0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s0}")
    # the input generator's spawn placement (plain C, no device code)
    place = os.path.join(LIBDIR, "libplace.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    os.path.join(HERE, "placement.c"), "-o", place + ".tmp"], check=True)
    os.replace(place + ".tmp", place)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    # the manifest the binding checks the sources against when it loads the
    # library: a library built from other sources is refused
    with open(MANIFEST + ".tmp", "w") as f:
        json.dump({"library": os.path.basename(LIB), "sources": digests}, f, indent=1, sort_keys=True)
    os.replace(MANIFEST + ".tmp", MANIFEST)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
