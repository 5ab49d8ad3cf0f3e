"""Pins of the oracle's KMC bookkeeping (oracle/kmc.py): the lattice proposal
set of App. C and the event selection of Alg. 1 (Sec. 2.1), CPU only.

* Targets and masks against brute force on positions: each hop is applied to
  the charge's coordinates in floating point, wrapped by the box length (or
  checked against the box in free space) and looked up in a set of occupied
  positions; the oracle works on integer site indices instead.
* Selection against hand-computed cumulative sums, the beta = 0 closed form
  (every valid slot has rate nu, so T = Q zeta selects valid slot
  ceil(V zeta) - 1), and the fraction of a uniform grid of T that each slot
  takes (r_j / Q exactly).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def brute_targets(xyz, n, offsets, periodic):
    occ = {tuple(p) for p in np.asarray(xyz).tolist()}
    N, K = len(xyz), len(offsets)
    valid = np.zeros((N, K), bool)
    tpos = np.zeros((N, K, 3))
    for i in range(N):
        for k in range(K):
            p = [xyz[i][d] + float(offsets[k][d]) for d in range(3)]
            if periodic:
                p = [v - n * math.floor(v / n) for v in p]
                inside = True
            else:
                inside = all(0.0 < v < n for v in p)
            tpos[i, k] = p
            valid[i, k] = inside and tuple(p) not in occ
    return tpos, valid


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("hops", ["6", "14", "26"])
def test_lattice_targets_match_brute_force(periodic, hops):
    n, N = 5, 60
    sites, xyz, q = W.lattice_charges(n, N, 31)
    off = W.hops(hops)
    t, v = O.lattice_targets(sites, n, off, periodic)
    tpos, vb = brute_targets(xyz, n, off, periodic)
    np.testing.assert_array_equal(v, vb)
    np.testing.assert_array_equal(W.site_xyz(t[v], n), tpos[vb])


def test_full_lattice_has_no_valid_slot():
    n = 4
    sites = np.arange(n ** 3)
    for periodic in (False, True):
        _, v = O.lattice_targets(sites, n, W.HOPS26, periodic)
        assert not v.any()


def test_selection_intervals_by_hand():
    # rates 1, 0 (masked), 2, 0.5: R = 1, 1, 3, 3.5
    r = np.array([1.0, 0.0, 2.0, 0.5])
    assert list(O.cumulative(r)) == [1.0, 1.0, 3.0, 3.5]
    cases = {0.25: 0, 1.0: 0, 1.0 + 1e-12: 2, 2.999: 2, 3.0: 2, 3.2: 3, 3.5: 3}
    for T, j in cases.items():
        assert O.select_slot(r, T) == j, T
    assert O.select_slot(r, 3.6) == -1
    assert O.select_slot(np.zeros(5), 0.0) == -1


def test_selection_fractions_are_rate_over_total():
    r = np.array([0.5, 0.0, 1.25, 0.25, 2.0])
    Q = r.sum()
    m = 40000
    T = Q * (np.arange(m) + 0.5) / m
    counts = np.bincount([O.select_slot(r, t) for t in T], minlength=len(r))
    np.testing.assert_allclose(counts / m, r / Q, atol=1.0 / m)


def test_zero_beta_is_a_uniform_choice():
    rng = np.random.default_rng(3)
    dU = rng.normal(size=200)
    valid = rng.random(200) < 0.6
    V = int(valid.sum())
    for kind in (1, 2):
        r = O.propensities(kind, 3.0, 0.0, dU, valid)
        assert np.all(r[valid] == 3.0) and np.all(r[~valid] == 0.0)
        for zeta in (1e-9, 0.3, 0.77, 1.0):
            j = O.select_slot(r, 3.0 * V * zeta)
            assert j == np.nonzero(valid)[0][math.ceil(V * zeta) - 1]
    assert O.time_increment(6.0, math.exp(-3.0)) == pytest.approx(0.5)


def test_rate_kinds():
    dU = np.array([-1.0, 0.0, 0.7, -1e4])
    valid = np.array([True, True, True, False])
    r1 = O.propensities(1, 2.0, 1.5, dU, valid)
    np.testing.assert_allclose(r1[:3], 2.0 * np.exp(-1.5 * dU[:3]), rtol=1e-15)
    r2 = O.propensities(2, 2.0, 1.5, dU, valid)
    np.testing.assert_allclose(r2[:3], [2.0, 2.0, 2.0 * math.exp(-1.05)], rtol=1e-15)
    assert r1[3] == 0.0 and r2[3] == 0.0
    # the exponent cap keeps very favourable hops finite
    assert O.propensities(1, 1.0, 1.0, np.array([-1e4]), np.array([True]))[0] == pytest.approx(math.exp(600.0))
