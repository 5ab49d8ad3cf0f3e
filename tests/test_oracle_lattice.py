"""Pins of the oracle's periodic lattice sums (CPU only).

The oracle sums Y_s^t(nu)/|nu|^{s+1} over complete cubic shells of
V_inf = Z^3 minus {|nu_k| <= 1} and removes the tail by Richardson
extrapolation (brute force).  Here the same sums are evaluated by a different
method written independently in the test: the Ewald split of the lattice sum of
a homogeneous harmonic polynomial (real-space incomplete-gamma sum plus a
reciprocal-space Gaussian sum, Hecke-Bochner), minus the 26 copies of V_box,
with harmonics from scipy.  Also checked: the zero pattern cubic symmetry
forces (odd s; t not a multiple of 4) and the closed-form V_box constant
(6 + 8/sqrt(3) + 12/sqrt(2)) ~ 19.104 printed in Sec. 3.1.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle as O


def Y_classical(n, m, theta, phi):
    """sqrt((n-|m|)!/(n+|m|)!) P_n^{|m|}(cos t) e^{i m p} without Condon-Shortley phase, from scipy"""
    y = sp.sph_harm_y(n, m, theta, phi) * math.sqrt(4 * math.pi / (2 * n + 1))
    return y * ((-1) ** m if m > 0 else 1)


def solid(s, t, v):
    """homogeneous harmonic polynomial |v|^s Y_s^t(angles of v)"""
    r = np.linalg.norm(v)
    return r ** s * Y_classical(s, t, math.acos(v[2] / r), math.atan2(v[1], v[0]))


def ewald_lattice_sum(s, t, alpha=math.sqrt(math.pi), nmax=6):
    g = math.gamma(s + 0.5)
    total = 0.0 + 0.0j
    rng = range(-nmax, nmax + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                if i == j == k == 0:
                    continue
                v = np.array([i, j, k], float)
                rr = float(v @ v)
                P = solid(s, t, v)
                total += P * sp.gammaincc(s + 0.5, alpha * alpha * rr) / rr ** (s + 0.5)
                total += ((-1j) ** s) * P * math.pi ** (s - 0.5) / g * math.exp(-math.pi ** 2 * rr / alpha ** 2) / rr
    box = sum(solid(s, t, np.array([i, j, k], float)) / (i * i + j * j + k * k) ** (s + 0.5)
              for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1) if (i, j, k) != (0, 0, 0))
    return total - box


@pytest.fixture(scope="module")
def lam():
    return O.lattice_sums(24)


@pytest.mark.parametrize("s,t", [(4, 0), (4, 4), (4, -4), (6, 0), (6, 4), (8, 0), (8, 8), (10, 4), (12, 12),
                                 (16, 8), (20, 0), (24, 20)])
def test_lattice_sums_match_ewald_split(lam, s, t):
    ref = ewald_lattice_sum(s, t)
    got = lam[O.idx(s, t)]
    # absolute floor: rounding of terms of size up to 1 (the nearest copies) in the sums
    assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-14


def test_lattice_sum_zero_pattern(lam):
    big = np.max(np.abs(lam))
    for s in range(25):
        for t in range(-s, s + 1):
            v = lam[O.idx(s, t)]
            if s % 2 == 1 or s < 3:
                assert v == 0
            elif t % 4 != 0:
                assert abs(v) < 1e-13 * big


def test_vbox_constant_closed_form():
    # Sec. 3.1: sum over the 26 neighbouring copies of 1/|nu| = 6 + 8/sqrt(3) + 12/sqrt(2) ~ 19.104
    s = sum(1.0 / math.sqrt(i * i + j * j + k * k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
            if (i, j, k) != (0, 0, 0))
    assert s == pytest.approx(6 + 8 / math.sqrt(3) + 12 / math.sqrt(2), rel=1e-15)
    assert round(s, 3) == 19.104
