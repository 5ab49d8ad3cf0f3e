"""Pins of O-exact: direct pair sums and tin-foil Ewald sums (CPU only).

* Madelung constants of rock salt and caesium chloride (tests/golden/madelung.json).
* The Ewald energy does not depend on the splitting parameter alpha.
* dU of a move equals the difference of two total energies, for both sums
  (different code paths: per-pair potential vs. pair sum with self terms).
* A hop by a whole period changes nothing; dU of a target on another charge is NaN.
* The conducting-surroundings convention against brute force: summing the
  copies of a neutral pair over growing cubes gives the Ewald energy plus
  (2 pi / 3V)|M|^2 (the surface term that the dipole correction of App. B removes).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "madelung.json")))


def test_madelung_rock_salt():
    na = [(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0)]
    cl = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)]
    xyz = np.array(na + cl, float) + 0.25
    q = np.array([1.0] * 4 + [-1.0] * 4)
    U = O.ewald_energy(xyz, q, 2.0)
    assert U / 4 == pytest.approx(-GOLD["NaCl"], rel=1e-13)


def test_madelung_caesium_chloride():
    xyz = np.array([[0.1, 0.2, 0.3], [0.6, 0.7, 0.8]])
    q = np.array([1.0, -1.0])
    U = O.ewald_energy(xyz, q, 1.0)
    assert U == pytest.approx(-GOLD["CsCl"] / (math.sqrt(3) / 2), rel=1e-13)


def random_box(seed, N=12, a=5.0):
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0, a, size=(N, 3))
    q = np.array([1.0, -1.0] * (N // 2))
    return xyz, q, a


def test_ewald_independent_of_alpha():
    xyz, q, a = random_box(1)
    U1 = O.ewald_energy(xyz, q, a, *O.ewald_params(a, rc=0.5 * a))
    U2 = O.ewald_energy(xyz, q, a, *O.ewald_params(a, rc=0.3 * a))
    U3 = O.ewald_energy(xyz, q, a, *O.ewald_params(a, rc=0.9 * a))
    assert U1 == pytest.approx(U2, abs=1e-13 * len(q))
    assert U1 == pytest.approx(U3, abs=1e-13 * len(q))


def test_ewald_dU_is_energy_difference():
    xyz, q, a = random_box(2)
    idx = np.array([0, 3, 7])
    tgt = np.array([[1.0, 2.0, 3.0], [4.9, 0.1, 2.2], [0.3, 4.4, 4.8]])
    dU = O.ewald_dU(xyz, q, a, idx, tgt)
    U0 = O.ewald_energy(xyz, q, a)
    for s, i in enumerate(idx):
        x2 = xyz.copy()
        x2[i] = tgt[s]
        assert dU[s] == pytest.approx(O.ewald_energy(x2, q, a) - U0, abs=1e-12)


def test_direct_dU_is_energy_difference():
    xyz, q, _ = random_box(3, N=20)
    idx = np.array([1, 5, 19])
    tgt = np.array([[1.0, 2.0, 3.0], [4.9, 0.1, 2.2], [0.3, 4.4, 4.8]])
    dU = O.direct_dU(xyz, q, idx, tgt)
    U0 = O.direct_energy(xyz, q)
    for s, i in enumerate(idx):
        x2 = xyz.copy()
        x2[i] = tgt[s]
        assert dU[s] == pytest.approx(O.direct_energy(x2, q) - U0, abs=1e-12)


def test_periodic_hop_by_period_and_singular_target():
    xyz, q, a = random_box(4)
    dU = O.ewald_dU(xyz, q, a, [2, 2], [xyz[2] + [a, 0, -a], xyz[5] + [0, a, 0]])
    assert abs(dU[0]) < 1e-12
    assert np.isnan(dU[1])
    assert np.isnan(O.direct_dU(xyz, q, [2], [xyz[5]])[0])


def test_cubic_shell_sum_is_tinfoil_plus_surface_term():
    a = 4.0
    r1, r2 = np.array([0.7, 1.1, 2.3]), np.array([2.9, 0.4, 1.8])
    d = r1 - r2

    def shells(R):
        g = np.arange(-R, R + 1)
        nu = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(float)
        nu = nu[np.any(nu != 0, 1)]
        return np.sum(1 / np.linalg.norm(a * nu, axis=1) - 1 / np.linalg.norm(d + a * nu, axis=1)) - 1 / np.linalg.norm(d)

    Rs = np.array([20.0, 30.0, 40.0])
    A = np.stack([np.ones(3), Rs ** -2, Rs ** -4], 1)
    limit = np.linalg.solve(A, [shells(int(R)) for R in Rs])[0]
    Ue = O.ewald_energy(np.array([r1, r2]), np.array([1.0, -1.0]), a)
    surface = 2 * math.pi / (3 * a ** 3) * float(d @ d)
    assert limit == pytest.approx(Ue + surface, abs=1e-6)
    assert abs(limit - Ue) > 0.1  # the surface term is not negligible here


def test_periodic_self_change_caesium_chloride():
    """psi_self - psi(b) with b half the body diagonal is the energy per ion pair
    of caesium chloride (a + ion's interaction with its own lattice minus the
    - lattice at the body centres): -M_CsCl / r_nn, r_nn = a sqrt(3) / 2"""
    for a in (1.0, 7.0, 64.0):
        b = np.array([a / 2, a / 2, a / 2])
        want = -GOLD["CsCl"] / (a * math.sqrt(3.0) / 2.0)
        assert O.periodic_self_change(a, b) == pytest.approx(want, rel=1e-14)
        # periodic in the displacement
        assert O.periodic_self_change(a, b - np.array([a, 0, 2 * a])) == pytest.approx(want, rel=1e-14)


def test_periodic_self_change_small_displacement():
    """psi(d) = 1/|d| + psi_self + (2 pi / 3V)|d|^2 + O(|d|^4 / a^5) (the background
    makes the Laplacian of psi - 1/r equal 4 pi / V, isotropic by cubic
    symmetry): the remainder falls as |d|^4 along a fixed direction"""
    a = 10.0
    rem = []
    for dd in (0.25, 0.5, 1.0):
        d = dd * np.array([1.0, 2.0, 2.0]) / 3.0
        v = O.periodic_self_change(a, d)
        rem.append(v - (-1.0 / dd - 2.0 * math.pi / (3.0 * a ** 3) * dd * dd))
    assert abs(rem[0]) < 4.0 * 0.25 ** 4 / a ** 5
    assert rem[1] / rem[0] == pytest.approx(16.0, rel=0.02)
    assert rem[2] / rem[1] == pytest.approx(16.0, rel=0.02)


@pytest.mark.parametrize("n,N,hops", [(8, 100, "26"), (12, 300, "6"), (10, 500, "26")])
def test_lattice_ewald_matches_pair_ewald(n, N, hops):
    """The FFT lattice Ewald (reciprocal part by one 3-D FFT of the site charges)
    against the pair-by-pair Ewald sum (pinned by the Madelung constants), and
    independent of the splitting parameter"""
    sites, xyz, q = W.lattice_charges(n, N, 71 + n)
    t, v = O.lattice_targets(sites, n, W.hops(hops), True)
    v = v.reshape(-1)
    idx = np.repeat(np.arange(N), len(W.hops(hops)))[v][:150]
    ts = t.reshape(-1)[v][:150]
    a = O.LatticeEwald(sites, q, n).dU_many(idx, ts)
    b = O.ewald_dU(xyz, q, n, idx, W.site_xyz(ts, n))
    c = O.LatticeEwald(sites, q, n, alpha_h=0.2).dU_many(idx, ts)
    scale = np.mean(np.abs(b))
    assert np.max(np.abs(a - b)) < 1e-13 * scale
    assert np.max(np.abs(a - c)) < 1e-13 * scale
