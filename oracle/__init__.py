"""CPU oracle for FMM electrostatics in kinetic Monte Carlo (arXiv:1905.04065).

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 statement of what the method
computes, used to check the GPU library.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg import this package; the GPU library never
does, and the two share no code.

Two oracles:
  * O-exact: direct pair sums (free space) and tin-foil Ewald sums (periodic);
  * O-fmm:   the FMM-KMC algorithm of Sec. 3 step by step (class ``FmmKmc``).

Coefficient arrays are complex, indexed n*n + n + m, in the classical
normalisation Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^{|m|}(cos t) e^{i m p}.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build
from .ewald_lattice import LatticeEwald  # noqa: F401
from .kmc import cumulative, lattice_targets, propensities, select_slot, time_increment  # noqa: F401

_lib = None


def lib():
    global _lib
    if _lib is None:
        if _build.needs_build():
            _build.build()
        L = C.CDLL(_build.LIB)
        d, i, i64, vp = C.c_double, C.c_int, C.c_int64, C.c_void_p
        sig = {
            "or_sph_harmonics": (None, [i, d, d, vp]),
            "or_p2m": (None, [i, i, vp, vp, vp, vp]),
            "or_m2m": (None, [i, vp, vp, vp]),
            "or_m2l": (None, [i, vp, vp, vp]),
            "or_l2l": (None, [i, vp, vp, vp]),
            "or_p2l": (None, [i, d, vp, vp, vp]),
            "or_eval_multipole": (d, [i, vp, vp, vp]),
            "or_eval_local": (d, [i, vp, vp, vp]),
            "or_lattice_sums": (None, [i, vp]),
            "or_direct_energy": (d, [i, vp, vp]),
            "or_direct_dU": (None, [i, vp, vp, i, vp, vp, vp]),
            "or_ewald_energy": (d, [i, vp, vp, d, d, d, d]),
            "or_ewald_dU": (None, [i, vp, vp, d, d, d, d, i, vp, vp, vp]),
            "or_periodic_self_change": (d, [d, vp]),
            "of_set_self_image": (None, [vp, i]),
            "of_set_field": (None, [vp, vp]),
            "of_create": (vp, [i, d, i, i, i, vp, vp, i]),
            "of_create_levels": (vp, [i, d, i, i, i, vp, vp, i, i]),
            "of_destroy": (None, [vp]),
            "of_energy": (d, [vp]),
            "of_propose": (None, [vp, i, vp, vp, vp]),
            "of_accept": (d, [vp, i64, vp]),
            "of_nterms": (i, [vp]),
            "of_fine_cell_of": (i, [vp, vp]),
            "of_get_local": (None, [vp, i, vp]),
            "of_get_level_local": (None, [vp, i, i, vp]),
            "of_get_multipole": (None, [vp, i, i, vp]),
            "of_get_far": (None, [vp, vp, vp, vp]),
            "of_get_positions": (None, [vp, vp]),
            "of_potential": (d, [vp, vp, i64]),
            "of_rebuild_multipoles": (None, [vp, i, i, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def nterms(p):
    return (p + 1) * (p + 1)


def idx(n, m):
    return n * n + n + m


# ---- harmonics and single expansions -----------------------------------------

def sph_harmonics(nmax, theta, phi):
    out = np.zeros(nterms(nmax), np.complex128)
    lib().or_sph_harmonics(nmax, float(theta), float(phi), _p(out))
    return out


def p2m(p, xyz, q, c):
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q)
    c = _f64(c)
    out = np.zeros(nterms(p), np.complex128)
    lib().or_p2m(p, len(q), _p(xyz), _p(q), _p(c), _p(out))
    return out


def _op(name, p, O, Q):
    O = np.ascontiguousarray(O, np.complex128)
    Q = _f64(Q)
    out = np.zeros(nterms(p), np.complex128)
    getattr(lib(), name)(p, _p(O), _p(Q), _p(out))
    return out


def m2m(p, O, Q):
    """Q = old centre - new centre"""
    return _op("or_m2m", p, O, Q)


def m2l(p, O, Q):
    """Q = source centre - target centre"""
    return _op("or_m2l", p, O, Q)


def l2l(p, O, Q):
    """Q = old centre - new centre"""
    return _op("or_l2l", p, O, Q)


def p2l(p, q, src, c):
    out = np.zeros(nterms(p), np.complex128)
    lib().or_p2l(p, float(q), _p(_f64(src)), _p(_f64(c)), _p(out))
    return out


def eval_multipole(p, M, c, x):
    M = np.ascontiguousarray(M, np.complex128)
    return lib().or_eval_multipole(p, _p(M), _p(_f64(c)), _p(_f64(x)))


def eval_local(p, L, c, x):
    L = np.ascontiguousarray(L, np.complex128)
    return lib().or_eval_local(p, _p(L), _p(_f64(c)), _p(_f64(x)))


def lattice_sums(smax):
    out = np.zeros(nterms(smax), np.complex128)
    lib().or_lattice_sums(smax, _p(out))
    return out


# ---- O-exact -----------------------------------------------------------------

def direct_energy(xyz, q):
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q)
    return lib().or_direct_energy(len(q), _p(xyz), _p(q))


def direct_dU(xyz, q, idx_, tgt):
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q)
    idx_ = np.ascontiguousarray(idx_, np.int64)
    tgt = _f64(tgt, (-1, 3))
    out = np.zeros(len(idx_))
    lib().or_direct_dU(len(q), _p(xyz), _p(q), len(idx_), _p(idx_), _p(tgt), _p(out))
    return out


def ewald_params(a, rc=None, tol_digits=16.5):
    """alpha, rc, kc with erfc(alpha rc) and exp(-kc^2/4alpha^2) below 10^-tol"""
    if rc is None:
        rc = 0.5 * a
    x = 1.0
    while np.exp(-x * x) / x > 10.0 ** (-tol_digits):  # erfc(x) ~ exp(-x^2)/(x sqrt(pi))
        x += 0.01
    alpha = x / rc
    kc = 2.0 * alpha * x
    return alpha, rc, kc


def ewald_energy(xyz, q, a, alpha=None, rc=None, kc=None):
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q)
    if alpha is None:
        alpha, rc, kc = ewald_params(a, rc)
    return lib().or_ewald_energy(len(q), _p(xyz), _p(q), float(a), alpha, rc, kc)


def ewald_dU(xyz, q, a, idx_, tgt, alpha=None, rc=None, kc=None):
    xyz = _f64(xyz, (-1, 3))
    q = _f64(q)
    idx_ = np.ascontiguousarray(idx_, np.int64)
    tgt = _f64(tgt, (-1, 3))
    if alpha is None:
        alpha, rc, kc = ewald_params(a, rc)
    out = np.zeros(len(idx_))
    lib().or_ewald_dU(len(q), _p(xyz), _p(q), float(a), alpha, rc, kc, len(idx_), _p(idx_), _p(tgt),
                      _p(out))
    return out


def periodic_self_change(a, d):
    """psi_self - psi(d): a unit charge's interaction with its own periodic
    copies after a displacement d, minus before (tin-foil Ewald)"""
    return lib().or_periodic_self_change(float(a), _p(_f64(d)))


# ---- O-fmm -------------------------------------------------------------------

class FmmKmc:
    """Step-by-step FMM-KMC (Sec. 3) in FP64.

    bc: "free" or "periodic"; L: levels (root = 1); p: expansion order.
    lazy: form the fine-level local expansion of a cell only when a proposal or
    query needs it (same arithmetic, restricted to those cells).
    self_image: "expansion" (the paper's self terms of Sec. 3.1) or "exact"
    (q^2 (psi_self - psi(r' - r)), tin-foil Ewald).
    per_level: keep the local expansion of every level apart and update each
    level's interaction-list cells at an accept (instead of every fine cell).
    """

    def __init__(self, xyz, q, a, L, p, bc="free", lazy=False, self_image="expansion", per_level=False,
                 field=(0.0, 0.0, 0.0)):
        self.xyz = _f64(xyz, (-1, 3)).copy()
        self.q = _f64(q).copy()
        self.a, self.L, self.p = float(a), int(L), int(p)
        self.bc = bc
        if bc == "periodic" and L < 3:
            raise ValueError("periodic boxes need L >= 3")
        if bc == "periodic" and abs(self.q.sum()) > 1e-12:
            raise ValueError("periodic boxes must be neutral")
        self._c = lib().of_create_levels(1 if bc == "periodic" else 0, self.a, self.L, self.p, len(self.q),
                                         _p(self.xyz), _p(self.q), 1 if lazy else 0, 1 if per_level else 0)
        self.per_level = bool(per_level)
        if self_image not in ("expansion", "exact"):
            raise ValueError("self_image must be 'expansion' or 'exact'")
        # periodic boxes: the moving charge's own copies by the paper's terms
        # (V_box sum, constant, 1/2 dE.R'dK) or by the exact Ewald change
        lib().of_set_self_image(self._c, 1 if self_image == "exact" else 0)
        # uniform external field: -q E.d per hop (Sec. 6.3 applies one)
        lib().of_set_field(self._c, _p(_f64(field, (3,))))

    def close(self):
        if getattr(self, "_c", None):
            lib().of_destroy(self._c)
            self._c = None

    def __del__(self):
        self.close()

    @property
    def energy(self):
        return lib().of_energy(self._c)

    def propose(self, idx_, tgt):
        idx_ = np.ascontiguousarray(idx_, np.int64)
        tgt = _f64(tgt, (-1, 3))
        out = np.zeros(len(idx_))
        lib().of_propose(self._c, len(idx_), _p(idx_), _p(tgt), _p(out))
        return out

    def accept(self, i, newpos):
        return lib().of_accept(self._c, int(i), _p(_f64(newpos)))

    def positions(self):
        out = np.zeros((len(self.q), 3))
        lib().of_get_positions(self._c, _p(out))
        return out

    def level_local(self, level, cell):
        """Psi of one cell on a level (per-level expansions: that level's own terms)"""
        out = np.zeros(nterms(self.p), np.complex128)
        lib().of_get_level_local(self._c, int(level), int(cell), _p(out))
        return out

    def local(self, cell):
        out = np.zeros(nterms(self.p), np.complex128)
        lib().of_get_local(self._c, int(cell), _p(out))
        return out

    def multipole(self, level, cell):
        out = np.zeros(nterms(self.p), np.complex128)
        lib().of_get_multipole(self._c, int(level), int(cell), _p(out))
        return out

    def rebuilt_multipole(self, level, cell):
        out = np.zeros(nterms(self.p), np.complex128)
        lib().of_rebuild_multipoles(self._c, int(level), int(cell), _p(out))
        return out

    def far(self):
        E, K, H = (np.zeros(nterms(self.p), np.complex128) for _ in range(3))
        lib().of_get_far(self._c, _p(E), _p(K), _p(H))
        return E, K, H

    def fine_cell_of(self, x):
        return lib().of_fine_cell_of(self._c, _p(_f64(x)))

    def potential(self, x, exclude=-1):
        """potential at x from every charge except `exclude` (near + local + far)"""
        self.local(self.fine_cell_of(x))  # forms the cell's expansion if lazy
        return lib().of_potential(self._c, _p(_f64(x)), int(exclude))
