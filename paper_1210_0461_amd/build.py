"""Build the CRoP HIP library (libcrop.so) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcrop.so")
SOURCES = ["api.hip", "k_route.hip", "k_exact.hip", "k_result.hip", "k_topk.hip",
           "k_learned.hip", "batch.hip", "k_cs.hip", "predictor.hip", "k_sbroute.hip", "noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed fp32 instructions stay off: some of their forms are unreliable
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in parallel, then link the shared
    library.  Always compiles (no up-to-date check)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    t0 = time.time()
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


def _wait(item):
    src, p = item
    if p.wait() != 0:
        raise RuntimeError(f"hipcc failed on {src}")


if __name__ == "__main__":
    build(verbose=True)
