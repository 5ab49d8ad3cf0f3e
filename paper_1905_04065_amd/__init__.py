"""FMM electrostatics for kinetic Monte Carlo on AMD MI355X (gfx950).

Thin Python binding of the C-ABI in include/fmmkmc.h (libfmmkmc.so, built
in-tree by build_ext.py).  Python only marshals arguments: every step of the
computation runs in the library's HIP kernels.  PyTorch provides device memory
and the stream.  There is no fallback: if the library is missing or no GPU is
visible, using this package raises.

Method: Saunders, Grant, Mueller, Thompson, "Fast electrostatic solvers for
kinetic Monte Carlo simulations" (arXiv:1905.04065), Sec. 3.
"""
import ctypes as C
import os

import numpy as np

__all__ = ["Batch", "Context", "FmmKmcError", "Slab", "library_path", "load_library"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, EINVAL, EDOMAIN, ECOINCIDENT, ECAPACITY, ESTATE, EHIP, ENOMEM = range(8)
_NAMES = {EINVAL: "EINVAL", EDOMAIN: "EDOMAIN", ECOINCIDENT: "ECOINCIDENT", ECAPACITY: "ECAPACITY",
          ESTATE: "ESTATE", EHIP: "EHIP", ENOMEM: "ENOMEM"}


class FmmKmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("a", C.c_double), ("bc", C.c_int), ("levels", C.c_int), ("order", C.c_int),
                ("precision", C.c_int), ("lattice_n", C.c_int), ("cell_capacity", C.c_int),
                ("device", C.c_int), ("stream", C.c_void_p), ("self_image", C.c_int), ("per_level", C.c_int)]


_SELF_IMAGE = {"expansion": 0, "exact": 1}


def library_path():
    return os.path.join(_HERE, "libfmmkmc.so")


def load_library():
    """Load libfmmkmc.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1905_04065_amd/build_ext.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(path)
    vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
    sig = {
        "fmmkmc_create": (i32, [C.POINTER(_Params), i64, vp, vp, C.POINTER(vp)]),
        "fmmkmc_initialise": (i32, [vp, C.POINTER(d)]),
        "fmmkmc_propose": (i32, [vp, i64, vp, vp, vp, vp]),
        "fmmkmc_propose_noalloc": (i32, [vp, i64, vp, vp, vp, vp]),
        "fmmkmc_propose_dats": (i32, [vp, i32, vp, i32, vp, vp, vp, vp]),
        "fmmkmc_propose_lattice": (i32, [vp, i32, vp, vp, vp]),
        "fmmkmc_accept": (i32, [vp, i64, vp, C.POINTER(d)]),
        "fmmkmc_energy": (i32, [vp, C.POINTER(d)]),
        "fmmkmc_positions": (i32, [vp, vp]),
        "fmmkmc_potential": (i32, [vp, i64, vp, vp, vp]),
        "fmmkmc_multipole": (i32, [vp, i32, i64, vp]),
        "fmmkmc_set_field": (i32, [vp, vp]),
        "fmmkmc_set_profiling": (i32, [vp, i32]),
        "fmmkmc_kernel_time": (i32, [vp, C.c_char_p, C.POINTER(d), C.POINTER(i64)]),
        "fmmkmc_last_error": (C.c_char_p, [vp]),
        "fmmkmc_destroy": (i32, [vp]),
        "fmmkmc_batch_create": (i32, [i32, vp, i32, vp, vp, C.POINTER(vp)]),
        "fmmkmc_batch_set_rates": (i32, [vp, i32, d, d]),
        "fmmkmc_batch_step": (i32, [vp, i32, vp, vp, vp, vp, vp]),
        "fmmkmc_batch_proposals": (i32, [vp, i32, vp, vp]),
        "fmmkmc_batch_tune": (i32, [vp, i32]),
        "fmmkmc_batch_info": (i32, [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]),
        "fmmkmc_batch_set_profiling": (i32, [vp, i32]),
        "fmmkmc_batch_kernel_time": (i32, [vp, C.c_char_p, C.POINTER(d), C.POINTER(i64)]),
        "fmmkmc_batch_last_error": (C.c_char_p, [vp]),
        "fmmkmc_batch_destroy": (i32, [vp]),
        "fmmkmc_slab_create": (i32, [C.POINTER(_Params), i64, vp, vp, d, C.POINTER(vp)]),
        "fmmkmc_slab_initialise": (i32, [vp, C.POINTER(d)]),
        "fmmkmc_slab_propose_lattice": (i32, [vp, i32, vp, vp, vp]),
        "fmmkmc_slab_accept": (i32, [vp, i64, vp, C.POINTER(d)]),
        "fmmkmc_slab_energy": (i32, [vp, C.POINTER(d)]),
        "fmmkmc_slab_positions": (i32, [vp, vp]),
        "fmmkmc_slab_last_error": (C.c_char_p, [vp]),
        "fmmkmc_slab_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("fmmkmc needs a GPU: torch.cuda.is_available() is False")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _host_f64(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a.reshape(shape)


class Context:
    """One FMM-KMC system on one GPU (the KMCFMM object of Sec. 5.2).

    bc: "free" or "periodic"; levels: L (root = 1); order: p;
    precision: "fp64" or "mixed"; lattice_n: n > 0 when every charge sits on a
    site of the n^3 lattice of spacing a/n (enables propose_lattice);
    self_image (periodic): "expansion" (the self terms of Sec. 3.1) or "exact"
    (their exact Ewald value, see fmmkmc_params in include/fmmkmc.h);
    per_level: keep the local expansions of every level apart, so that an
    accept updates only the cells whose interaction lists hold the moved
    charge instead of every fine cell.
    """

    def __init__(self, xyz, q, a, levels, order, bc="free", precision="fp64", lattice_n=0, cell_capacity=0,
                 device=0, stream=None, self_image="expansion", per_level=False):
        torch = _torch()
        self._L = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        xyz = _host_f64(xyz, (-1, 3))
        q = _host_f64(q, (-1,))
        if len(q) != len(xyz):
            raise ValueError("xyz and q lengths differ")
        self.N = len(q)
        self.K = None
        prm = _Params(float(a), 1 if bc == "periodic" else 0, int(levels), int(order),
                      1 if precision == "mixed" else 0, int(lattice_n), int(cell_capacity), int(device),
                      C.c_void_p(stream.cuda_stream), _SELF_IMAGE[self_image], 1 if per_level else 0)
        h = C.c_void_p()
        rc = self._L.fmmkmc_create(C.byref(prm), self.N, xyz.ctypes.data_as(C.c_void_p),
                                   q.ctypes.data_as(C.c_void_p), C.byref(h))
        if rc != OK:
            raise FmmKmcError(rc, self._L.fmmkmc_last_error(None).decode())
        self._h = h
        self.a, self.bc, self.levels, self.order = float(a), bc, int(levels), int(order)
        self.precision, self.lattice_n = precision, int(lattice_n)
        self.self_image = self_image
        self.per_level = bool(per_level)

    # -- helpers --
    def _check(self, rc):
        if rc != OK:
            raise FmmKmcError(rc, self._L.fmmkmc_last_error(self._h).decode())

    def _dev(self, t, dtype):
        torch = _torch()
        t = torch.as_tensor(t, dtype=dtype, device=self.device)
        return t.contiguous()

    def close(self):
        if getattr(self, "_h", None):
            self._L.fmmkmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- API --
    def initialise(self):
        """Build the expansions; returns the total energy (Alg. fmm + fmm_evaluation)."""
        U = C.c_double()
        self._check(self._L.fmmkmc_initialise(self._h, C.byref(U)))
        return U.value

    def propose(self, idx, offs, targets, dU=None, check=True):
        """propose(P) of Sec. 5.2.1 in CSR form: charge idx[g] to targets[offs[g]:offs[g+1]]."""
        torch = _torch()
        idx = self._dev(idx, torch.int64)
        offs = self._dev(offs, torch.int64)
        targets = self._dev(targets, torch.float64).reshape(-1, 3)
        S = targets.shape[0]
        if dU is None:
            dU = torch.empty(S, dtype=torch.float64, device=self.device)
        rc = self._L.fmmkmc_propose(self._h, idx.numel(), _ptr(idx), _ptr(offs), _ptr(targets), _ptr(dU))
        if check:
            self._check(rc)
        return dU if check else (dU, rc)

    def propose_noalloc(self, idx, offs, targets, dU, check=True):
        """propose() through the allocation-free entry point: every array (device
        tensors idx, offs, targets, dU) is supplied by the caller"""
        rc = self._L.fmmkmc_propose_noalloc(self._h, idx.numel(), _ptr(idx), _ptr(offs), _ptr(targets), _ptr(dU))
        if check:
            self._check(rc)
        return rc

    def propose_pairs(self, idx, targets, check=True):
        """one target per charge index (a CSR with groups of one)"""
        torch = _torch()
        idx = self._dev(idx, torch.int64).reshape(-1)
        offs = torch.arange(idx.numel() + 1, dtype=torch.int64, device=self.device)
        return self.propose(idx, offs, targets, check=check)

    def propose_dats(self, K, C_, T, R, M, U=None, check=True):
        """propose_with_dats(C, T, R, M, U) of App. C."""
        torch = _torch()
        Ch = np.ascontiguousarray(np.asarray(C_, dtype=np.int32))
        T = self._dev(T, torch.int32)
        R = self._dev(R, torch.float64)
        M = self._dev(M, torch.uint8)
        if U is None:
            U = torch.empty(self.N * K, dtype=torch.float64, device=self.device)
        rc = self._L.fmmkmc_propose_dats(self._h, int(K), Ch.ctypes.data_as(C.c_void_p), len(Ch), _ptr(T), _ptr(R),
                                         _ptr(M), _ptr(U))
        if check:
            self._check(rc)
        return U.reshape(self.N, K) if check else (U.reshape(self.N, K), rc)

    def propose_lattice(self, offsets, dU=None, mask=None, want_mask=True):
        """dU[i, k] for the hop of charge i by offsets[k] (lattice mode); asynchronous."""
        torch = _torch()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
        K = off.shape[0]
        if dU is None:
            dU = torch.empty((self.N, K), dtype=torch.float64, device=self.device)
        if mask is None and want_mask:
            mask = torch.empty((self.N, K), dtype=torch.uint8, device=self.device)
        self._check(self._L.fmmkmc_propose_lattice(self._h, K, off.ctypes.data_as(C.c_void_p), _ptr(dU),
                                                   _ptr(mask) if mask is not None else None))
        return dU, mask

    def accept(self, i, pos):
        """accept((i, r')) of Sec. 5.2.2; returns dU of the move."""
        p = _host_f64(pos, (3,))
        dU = C.c_double()
        self._check(self._L.fmmkmc_accept(self._h, int(i), p.ctypes.data_as(C.c_void_p), C.byref(dU)))
        return dU.value

    @property
    def energy(self):
        U = C.c_double()
        self._check(self._L.fmmkmc_energy(self._h, C.byref(U)))
        return U.value

    def positions(self):
        torch = _torch()
        out = torch.empty((self.N, 3), dtype=torch.float64, device=self.device)
        self._check(self._L.fmmkmc_positions(self._h, _ptr(out)))
        return out

    def potential(self, xyz, exclude=None):
        torch = _torch()
        xyz = self._dev(xyz, torch.float64).reshape(-1, 3)
        m = xyz.shape[0]
        out = torch.empty(m, dtype=torch.float64, device=self.device)
        ex = None
        if exclude is not None:
            ex = self._dev(exclude, torch.int64).reshape(-1)
        self._check(self._L.fmmkmc_potential(self._h, m, _ptr(xyz), _ptr(ex) if ex is not None else None, _ptr(out)))
        return out

    def set_field(self, E):
        """uniform external field: every hop adds -q E.d (see fmmkmc_set_field)"""
        e = _host_f64(E, (3,))
        self._check(self._L.fmmkmc_set_field(self._h, e.ctypes.data_as(C.c_void_p)))

    def multipole(self, level, cell):
        """Phi of one octree cell in the library's real storage ((p+1)^2 doubles, see
        fmmkmc_multipole in include/fmmkmc.h)"""
        out = np.zeros((self.order + 1) ** 2)
        self._check(self._L.fmmkmc_multipole(self._h, int(level), int(cell), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_profiling(self, on=True):
        self._check(self._L.fmmkmc_set_profiling(self._h, 1 if on else 0))

    def kernel_time(self, name):
        """(total ms, launches) of a kernel since profiling was switched on"""
        ms, n = C.c_double(), C.c_int64()
        self._check(self._L.fmmkmc_kernel_time(self._h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Batch:
    """Replicas (initialised lattice-mode Contexts with one order and precision)
    advanced together: each KMC step is one launch per phase over all of them,
    replayed from a captured HIP graph.  The contexts stay owned by the caller."""

    def __init__(self, contexts, offsets, stream=None):
        torch = _torch()
        self._L = load_library()
        self.contexts = list(contexts)
        self.R = len(self.contexts)
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
        self.K = off.shape[0]
        self.device = self.contexts[0].device
        arr = (C.c_void_p * self.R)(*[c._h.value for c in self.contexts])
        st = C.c_void_p(stream.cuda_stream) if stream is not None else None
        h = C.c_void_p()
        rc = self._L.fmmkmc_batch_create(self.R, C.cast(arr, C.c_void_p), self.K, off.ctypes.data_as(C.c_void_p),
                                         st, C.byref(h))
        if rc != OK:
            raise FmmKmcError(rc, self._L.fmmkmc_batch_last_error(None).decode())
        self._h = h
        self._torch = torch

    def _check(self, rc):
        if rc != OK:
            raise FmmKmcError(rc, self._L.fmmkmc_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.fmmkmc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    rate_kind = 0

    def set_rates(self, kind, nu=1.0, beta=1.0):
        """propensity of a hop: 0 uniform over valid hops, 1 nu exp(-beta dU),
        2 nu min(1, exp(-beta dU))"""
        self._check(self._L.fmmkmc_batch_set_rates(self._h, int(kind), float(nu), float(beta)))
        self.rate_kind = int(kind)

    def step(self, u, with_dt=False):
        """KMC steps with the uniforms u: n_steps x R (rate kind 0) or
        n_steps x R x 2 (kinds 1, 2: zeta, xi per replica and step); returns
        device tensors (moved charge, new site, dU[, dt]), each n_steps x R."""
        torch = self._torch
        per = 1 if self.rate_kind == 0 else 2
        u = torch.as_tensor(u, dtype=torch.float64, device=self.device).reshape(-1, self.R * per).contiguous()
        n = u.shape[0]
        moved = torch.empty((n, self.R), dtype=torch.int64, device=self.device)
        site = torch.empty((n, self.R), dtype=torch.int64, device=self.device)
        dU = torch.empty((n, self.R), dtype=torch.float64, device=self.device)
        dt = torch.empty((n, self.R), dtype=torch.float64, device=self.device)
        self._check(self._L.fmmkmc_batch_step(self._h, n, _ptr(u), _ptr(moved), _ptr(site), _ptr(dU), _ptr(dt)))
        return (moved, site, dU, dt) if with_dt else (moved, site, dU)

    def proposals(self, r):
        """dU and mask (N_r x K device tensors) of replica r's last proposal pass"""
        torch = self._torch
        N = self.contexts[r].N
        dU = torch.empty((N, self.K), dtype=torch.float64, device=self.device)
        mask = torch.empty((N, self.K), dtype=torch.uint8, device=self.device)
        self._check(self._L.fmmkmc_batch_proposals(self._h, int(r), _ptr(dU), _ptr(mask)))
        return dU, mask

    def tune(self, rounds=5):
        self._check(self._L.fmmkmc_batch_tune(self._h, int(rounds)))
        return self.info()

    def info(self):
        slots, tile, blk = C.c_int64(), C.c_int(), C.c_int()
        self._check(self._L.fmmkmc_batch_info(self._h, C.byref(slots), C.byref(tile), C.byref(blk)))
        return {"slots_per_step": slots.value, "slot_tile": tile.value, "sweep_block": blk.value}

    def set_profiling(self, on=True):
        self._check(self._L.fmmkmc_batch_set_profiling(self._h, 1 if on else 0))

    def kernel_time(self, name):
        ms, n = C.c_double(), C.c_int64()
        self._check(self._L.fmmkmc_batch_kernel_time(self._h, name.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Slab:
    """Charges between two grounded plates (potential 0 at z = 0 and z = a/2),
    periodic in x and y, in a uniform field ez along z (Sec. 2.2.2 Dirichlet
    boundaries, by the first mirror image and the periodic algorithm)."""

    def __init__(self, xyz, q, a, levels, order, lattice_n, ez=0.0, precision="fp64", cell_capacity=0, device=0,
                 stream=None, self_image="expansion", per_level=False):
        torch = _torch()
        self._L = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        xyz = _host_f64(xyz, (-1, 3))
        q = _host_f64(q, (-1,))
        if len(q) != len(xyz):
            raise ValueError("xyz and q lengths differ")
        self.N = len(q)
        prm = _Params(float(a), 1, int(levels), int(order), 1 if precision == "mixed" else 0, int(lattice_n),
                      int(cell_capacity), int(device), C.c_void_p(stream.cuda_stream), _SELF_IMAGE[self_image],
                      1 if per_level else 0)
        h = C.c_void_p()
        rc = self._L.fmmkmc_slab_create(C.byref(prm), self.N, xyz.ctypes.data_as(C.c_void_p),
                                        q.ctypes.data_as(C.c_void_p), float(ez), C.byref(h))
        if rc != OK:
            raise FmmKmcError(rc, self._L.fmmkmc_slab_last_error(None).decode())
        self._h = h
        self.a, self.lattice_n, self.ez = float(a), int(lattice_n), float(ez)

    def _check(self, rc):
        if rc != OK:
            raise FmmKmcError(rc, self._L.fmmkmc_slab_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.fmmkmc_slab_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def initialise(self):
        U = C.c_double()
        self._check(self._L.fmmkmc_slab_initialise(self._h, C.byref(U)))
        return U.value

    def propose_lattice(self, offsets):
        """dU and mask (N x K device tensors) of every hop of every charge"""
        torch = _torch()
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
        K = off.shape[0]
        dU = torch.empty((self.N, K), dtype=torch.float64, device=self.device)
        mask = torch.empty((self.N, K), dtype=torch.uint8, device=self.device)
        self._check(self._L.fmmkmc_slab_propose_lattice(self._h, K, off.ctypes.data_as(C.c_void_p), _ptr(dU),
                                                        _ptr(mask)))
        return dU, mask

    def accept(self, i, new_xyz):
        p = np.ascontiguousarray(np.asarray(new_xyz, dtype=np.float64).reshape(3))
        d = C.c_double()
        self._check(self._L.fmmkmc_slab_accept(self._h, int(i), p.ctypes.data_as(C.c_void_p), C.byref(d)))
        return d.value

    @property
    def energy(self):
        U = C.c_double()
        self._check(self._L.fmmkmc_slab_energy(self._h, C.byref(U)))
        return U.value

    def positions(self):
        torch = _torch()
        out = torch.empty((self.N, 3), dtype=torch.float64, device=self.device)
        self._check(self._L.fmmkmc_slab_positions(self._h, _ptr(out)))
        return out
