"""Build libkepler.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_0812_2976_amd.build [-v]

Packed FP32 instructions are disabled (-packed-fp32-ops): the kernels are
written in scalar FP32 and the compiler is not allowed to pair them.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libkepler.so")
SOURCES = ["kep_kernels.hip", "kep_adjoint.hip", "kep_demc.hip", "kep_astro.hip", "kep_gn.hip", "kep_ragged64.hip",
           "kep_api.cpp"]
# Per-source flags.  The Gauss-Newton kernel's matrix products accumulate in
# ordinary VGPRs (gfx950 allows it): without this the compiler moves the
# accumulators to AGPRs and back around every unrolled group of products and
# waits for the products to finish each time.
EXTRA = {"kep_gn.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
ARCH = os.environ.get("KEP_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for src in SOURCES:           # the sources compile independently: in parallel
        obj = os.path.join(bdir, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [hipcc()] + flags() + EXTRA.get(src, []) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
