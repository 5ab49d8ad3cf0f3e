"""The C-ABI library loads and exports every entry point include/fmmkmc.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmmkmc.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(fmmkmc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_paper_interface():
    names = declared()
    for n in ("fmmkmc_create", "fmmkmc_initialise", "fmmkmc_propose", "fmmkmc_propose_dats",
              "fmmkmc_propose_lattice", "fmmkmc_accept", "fmmkmc_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1905_04065_amd as pkg
    path = pkg.library_path()
    if not os.path.exists(path):
        pytest.skip("libfmmkmc.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads_and_reports_create_errors_without_gpu():
    import paper_1905_04065_amd as pkg
    if not os.path.exists(pkg.library_path()):
        pytest.skip("libfmmkmc.so not built")
    L = pkg.load_library()
    # invalid parameters are rejected before any device work
    prm = pkg._Params(-1.0, 0, 3, 4, 0, 0, 0, 0, None)
    h = ctypes.c_void_p()
    xyz = (ctypes.c_double * 3)(0.5, 0.5, 0.5)
    q = (ctypes.c_double * 1)(1.0)
    rc = L.fmmkmc_create(ctypes.byref(prm), 1, ctypes.cast(xyz, ctypes.c_void_p), ctypes.cast(q, ctypes.c_void_p),
                         ctypes.byref(h))
    assert rc == pkg.EINVAL
    assert b"box side" in L.fmmkmc_last_error(None)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
