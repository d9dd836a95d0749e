"""Build libdgweno.so (HIP, gfx950) in-tree.

    python -m paper_2309_12019_amd.build

Compiles the stage kernels once per (dimension, degree) pair in parallel, the
C-ABI layer, and links them into paper_2309_12019_amd/libdgweno.so.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdgweno.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("DGWENO_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-fconstexpr-steps=100000000",
    # packed FP32 instructions stay off (the library computes in FP64 anyway)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + p.stdout[-8000:])
    return p.stdout


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    steps = []
    objs = []
    for dim in (1, 2):
        for p in (1, 2, 3, 4):
            o = os.path.join(BUILD, f"stage_{dim}_{p}.o")
            objs.append(o)
            steps.append([cc, *FLAGS, f"-DDGK_DIM={dim}", f"-DDGK_P={p}", "-c",
                          os.path.join(CSRC, "dg_stage.hip"), "-o", o])
    for name in ("dg_api", "dg_batch", "dg_util"):
        o = os.path.join(BUILD, f"{name}.o")
        objs.append(o)
        steps.append([cc, *FLAGS, "-c", os.path.join(CSRC, f"{name}.hip"), "-o", o])
    jobs = jobs or min(9, os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for out in ex.map(_run, steps):
            if verbose and out.strip():
                print(out)
    tmp = OUT + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
