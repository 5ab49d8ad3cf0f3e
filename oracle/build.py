"""Build the CPU oracle (plain C + OpenMP) into oracle/_build/.

Test infrastructure only: the oracle is loaded by the test suite, the smoke
check and the CPU-baseline leg of the benchmark, never by the GPU library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["harmonics.c", "expansions.c", "lattice.c", "exact.c", "fmm_kmc.c"]
LIB = os.path.join(HERE, "_build", "liboracle_fmmkmc.so")


def build(verbose=False):
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + ["oracle.h", "oracle_internal.h"]
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in deps)


if __name__ == "__main__":
    print(build(verbose=True))
