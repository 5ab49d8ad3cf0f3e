"""Compile the HIP library (csrc/*.hip) for gfx950 into libfmmkmc.so, in-tree.

Every translation unit is compiled separately (in parallel) and linked into
one shared library that exports the C-ABI of include/fmmkmc.h.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmmkmc.so")
ARCH = os.environ.get("FMMKMC_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}",
         # no packed FP32 instructions (v_pk_*_f32) anywhere
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def sources():
    return sorted(f for f in os.listdir(SRC) if f.endswith(".hip"))


def _compile(name, verbose):
    obj = os.path.join(OUT, name[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(SRC, name), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {name}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(OUT, exist_ok=True)
    names = sources()
    jobs = jobs or min(len(names), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda n: _compile(n, verbose), names))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
