"""Pins of the oracle's harmonics and expansion operators (CPU only).

Each check compares with something other than the oracle itself: closed forms
of low-degree harmonics, the Legendre addition theorem (via numpy's Legendre
polynomials), and direct Coulomb sums within the truncation bound of the
multipole / local expansions of Eq. (multipole_local_expansion).  M2M and L2L
of truncated expansions are exact, so those are checked to rounding.
"""
import math

import numpy as np
import pytest

import oracle as O


def sph(v):
    r = np.linalg.norm(v)
    return r, math.acos(v[2] / r), math.atan2(v[1], v[0])


def test_harmonics_closed_forms():
    th, ph = 0.7, -1.3
    Y = O.sph_harmonics(3, th, ph)
    c, s = math.cos(th), math.sin(th)
    assert Y[O.idx(0, 0)] == pytest.approx(1.0)
    assert Y[O.idx(1, 0)] == pytest.approx(c)
    assert Y[O.idx(1, 1)] == pytest.approx(s * np.exp(1j * ph) / math.sqrt(2.0))
    assert Y[O.idx(1, -1)] == pytest.approx(s * np.exp(-1j * ph) / math.sqrt(2.0))
    assert Y[O.idx(2, 0)] == pytest.approx((3 * c * c - 1) / 2)
    assert Y[O.idx(2, 2)] == pytest.approx(3 * s * s * np.exp(2j * ph) / math.sqrt(24.0))
    assert Y[O.idx(3, 0)] == pytest.approx((5 * c ** 3 - 3 * c) / 2)


@pytest.mark.parametrize("n", [0, 1, 4, 9, 17, 24])
def test_legendre_addition_theorem(n):
    rng = np.random.default_rng(n)
    t1, p1, t2, p2 = rng.uniform(0, math.pi), rng.uniform(-3, 3), rng.uniform(0, math.pi), rng.uniform(-3, 3)
    Y1 = O.sph_harmonics(n, t1, p1)
    Y2 = O.sph_harmonics(n, t2, p2)
    cosg = math.cos(t1) * math.cos(t2) + math.sin(t1) * math.sin(t2) * math.cos(p1 - p2)
    lhs = np.polynomial.legendre.legval(cosg, [0] * n + [1])
    rhs = sum(Y1[O.idx(n, -m)] * Y2[O.idx(n, m)] for m in range(-n, n + 1))
    assert abs(rhs.imag) < 1e-12
    assert rhs.real == pytest.approx(lhs, abs=1e-12)


def cluster(seed, k=6, radius=0.5, centre=(0.0, 0.0, 0.0)):
    rng = np.random.default_rng(seed)
    xyz = np.asarray(centre) + rng.uniform(-radius, radius, size=(k, 3)) / math.sqrt(3.0)
    q = rng.normal(size=k)
    return xyz, q


def direct(xyz, q, x):
    return float(np.sum(q / np.linalg.norm(np.asarray(x) - xyz, axis=1)))


@pytest.mark.parametrize("p", [2, 6, 12])
def test_p2m_within_truncation_bound(p):
    xyz, q = cluster(1)
    c = np.zeros(3)
    M = O.p2m(p, xyz, q, c)
    rho = np.max(np.linalg.norm(xyz - c, axis=1))
    for x in ([3.0, 0.4, -0.2], [0.0, 0.0, 2.0], [-1.5, -1.5, 1.0]):
        r = np.linalg.norm(x)
        bound = np.sum(np.abs(q)) / (r - rho) * (rho / r) ** (p + 1)
        err = abs(O.eval_multipole(p, M, c, x) - direct(xyz, q, x))
        assert err <= bound * 1.0001 + 1e-14


def test_p2m_converges_to_direct():
    xyz, q = cluster(2)
    x = [2.5, -1.0, 0.3]
    errs = [abs(O.eval_multipole(p, O.p2m(p, xyz, q, np.zeros(3)), np.zeros(3), x) - direct(xyz, q, x))
            for p in (4, 10, 20)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-12


@pytest.mark.parametrize("p", [3, 8, 12])
def test_m2m_exact(p):
    xyz, q = cluster(3, centre=(0.1, -0.2, 0.3))
    c1 = np.array([0.1, -0.2, 0.3])
    c2 = np.array([0.6, 0.3, -0.2])
    M1 = O.p2m(p, xyz, q, c1)
    M2 = O.m2m(p, M1, c1 - c2)
    ref = O.p2m(p, xyz, q, c2)
    assert np.max(np.abs(M2 - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("p", [4, 8, 12])
def test_m2l_within_bound(p):
    xyz, q = cluster(4)
    cs = np.zeros(3)
    ct = np.array([3.0, 1.0, -2.0])
    M = O.p2m(p, xyz, q, cs)
    L = O.m2l(p, M, cs - ct)
    a = np.max(np.linalg.norm(xyz - cs, axis=1))
    rng = np.random.default_rng(9)
    R = np.linalg.norm(ct - cs)
    for _ in range(5):
        y = ct + rng.uniform(-0.3, 0.3, size=3)
        b = np.linalg.norm(y - ct)
        # the local expansion of the truncated multipole converges at rate (a+b)/R
        bound = 2 * np.sum(np.abs(q)) / (R - a - b) * ((a + b) / R) ** (p + 1)
        err = abs(O.eval_local(p, L, ct, y) - direct(xyz, q, y))
        assert err <= bound


def test_m2l_converges_to_direct():
    xyz, q = cluster(5)
    ct = np.array([4.0, -1.0, 2.0])
    y = ct + np.array([0.2, -0.1, 0.25])
    errs = []
    for p in (5, 10, 20):
        L = O.m2l(p, O.p2m(p, xyz, q, np.zeros(3)), -ct)
        errs.append(abs(O.eval_local(p, L, ct, y) - direct(xyz, q, y)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-13


@pytest.mark.parametrize("p", [3, 8, 12])
def test_l2l_exact(p):
    xyz, q = cluster(6)
    ct = np.array([3.0, 2.0, -2.5])
    L = O.m2l(p, O.p2m(p, xyz, q, np.zeros(3)), -ct)
    c2 = ct + np.array([0.25, -0.25, 0.25])
    L2 = O.l2l(p, L, ct - c2)
    rng = np.random.default_rng(2)
    for _ in range(4):
        y = c2 + rng.uniform(-0.3, 0.3, size=3)
        assert O.eval_local(p, L2, c2, y) == pytest.approx(O.eval_local(p, L, ct, y), abs=1e-14)


@pytest.mark.parametrize("p", [4, 12])
def test_p2l_within_bound(p):
    src = np.array([2.0, -1.0, 1.5])
    c = np.array([0.1, 0.2, -0.1])
    L = O.p2l(p, -0.7, src, c)
    R = np.linalg.norm(src - c)
    for y in ([0.3, 0.0, 0.0], [0.0, -0.5, 0.4], [-0.3, 0.3, 0.3]):
        yy = c + np.array(y)
        b = np.linalg.norm(yy - c)
        bound = 0.7 / (R - b) * (b / R) ** (p + 1)
        err = abs(O.eval_local(p, L, c, yy) + 0.7 / np.linalg.norm(src - yy))
        assert err <= bound * 1.0001 + 1e-15
