"""Build step of the HIP library: compiles csrc/ for gfx950 into liblbm_axi.so (in-tree)."""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_axi.so")
SOURCES = ["lbm_kernels.hip", "lbm_axi.cpp", "eos_host.cpp", "scratch.hip"]
# No fast-math (the FP64 path is compared with an FP64 reference); multiply-adds are fused
# only within one expression (-ffp-contract=on), so that every kernel instantiation rounds
# the same arithmetic the same way; packed FP32 instructions are disabled.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-fno-fast-math", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall"]


def build(verbose: bool = False, jobs: int = 3) -> str:
    with tempfile.TemporaryDirectory(prefix="lbm_axi_build_") as tmp:
        procs, objs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = ["hipcc", *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
            objs.append(obj)
            if len(procs) >= jobs:
                if procs.pop(0).wait() != 0:
                    raise RuntimeError("hipcc failed")
        for p in procs:
            if p.wait() != 0:
                raise RuntimeError("hipcc failed")
        link = ["hipcc", "-shared", "--offload-arch=gfx950", *objs, "-o", LIB + ".tmp"]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
