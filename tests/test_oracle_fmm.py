"""Pins of O-fmm, the step-by-step FMM-KMC oracle (CPU only).

Against things other than O-fmm itself:
* free space with L <= 2 has empty interaction lists (Sec. 2.2.1), so every dU
  must equal the direct pair-sum dU of O-exact to rounding;
* free space at higher L: dU converges to O-exact as p grows, roughly a decade
  per three orders (Sec. 6.1);
* periodic: dU and the total energy converge to tin-foil Ewald (the dipole
  condition of Sec. 2.2.2 / App. B), which fixes the near-field self terms of
  Eq. (proposed_energy_sr), the V_box constant, the far-field factor 1/2 and
  the dipole correction together;
* invariants of the accept step: a round trip restores every local expansion
  and E, K, H to rounding; in free space dU(a->b) = -dU(b->a) after accepting
  a->b for a hop between neighbouring cells; the incrementally updated K equals
  the root multipole of a fresh upward pass;
* masked and singular proposals give NaN.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def lattice(n, N, seed):
    sites, xyz, q = W.lattice_charges(n, N, seed)
    return sites, xyz, q


def proposals(sites, n, periodic, hops=W.HOPS6):
    t, valid = W.lattice_targets(sites, n, hops, periodic)
    K = len(hops)
    idx = np.repeat(np.arange(len(sites)), K)
    tgt = W.site_xyz(t.reshape(-1), n)
    return idx, tgt, valid.reshape(-1)


def test_free_space_two_levels_is_direct_sum():
    n, N = 12, 60
    sites, xyz, q = lattice(n, N, 11)
    idx, tgt, valid = proposals(sites, n, False)
    f = O.FmmKmc(xyz, q, n, 2, 6, "free")
    d_fmm = f.propose(idx[valid], tgt[valid])
    d_dir = O.direct_dU(xyz, q, idx[valid], tgt[valid])
    assert np.max(np.abs(d_fmm - d_dir)) <= 1e-13 * np.max(np.abs(d_dir))
    assert f.energy == pytest.approx(O.direct_energy(xyz, q), abs=1e-12)


def test_free_space_converges_with_order():
    n, N = 16, 150
    sites, xyz, q = lattice(n, N, 12)
    idx, tgt, valid = proposals(sites, n, False)
    ref = O.direct_dU(xyz, q, idx[valid], tgt[valid])
    errs = []
    for p in (4, 7, 10, 13):
        d = O.FmmKmc(xyz, q, n, 4, p, "free").propose(idx[valid], tgt[valid])
        errs.append(np.mean(np.abs(d - ref)) / np.mean(np.abs(ref)))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3  # about a decade per +3 (Sec. 6.1); at least a factor 3
    assert errs[-1] < 1e-5


@pytest.fixture(scope="module")
def periodic_box():
    n, N = 8, 40
    sites, xyz, q = lattice(n, N, 13)
    idx, tgt, valid = proposals(sites, n, True)
    ref = O.ewald_dU(xyz, q, n, idx, tgt)
    Ue = O.ewald_energy(xyz, q, n)
    return n, xyz, q, idx, tgt, valid, ref, Ue


def test_periodic_matches_tinfoil_ewald(periodic_box):
    n, xyz, q, idx, tgt, valid, ref, Ue = periodic_box
    f = O.FmmKmc(xyz, q, n, 3, 18, "periodic")
    d = f.propose(idx, tgt)
    assert np.array_equal(np.isnan(d), ~valid)
    assert np.array_equal(np.isnan(ref), ~valid)
    assert np.max(np.abs(d[valid] - ref[valid])) < 2e-6 * np.mean(np.abs(ref[valid]))
    assert f.energy == pytest.approx(Ue, abs=1e-6)


def test_periodic_converges_with_order(periodic_box):
    n, xyz, q, idx, tgt, valid, ref, Ue = periodic_box
    errs = []
    for p in (6, 10, 14):
        d = O.FmmKmc(xyz, q, n, 3, p, "periodic").propose(idx[valid], tgt[valid])
        errs.append(np.max(np.abs(d - ref[valid])))
    assert errs[0] > 5 * errs[1] > 25 * errs[2]


def test_wrapped_and_unwrapped_targets_agree(periodic_box):
    n, xyz, q, idx, tgt, valid, ref, Ue = periodic_box
    f = O.FmmKmc(xyz, q, n, 3, 8, "periodic")
    sel = np.nonzero(valid)[0][:20]
    shift = np.array([n, -n, 2 * n], float)
    assert np.allclose(f.propose(idx[sel], tgt[sel]), f.propose(idx[sel], tgt[sel] + shift), atol=0, rtol=1e-13)


@pytest.mark.parametrize("bc", ["free", "periodic"])
def test_round_trip_restores_state(bc):
    n, N = 8, 40
    sites, xyz, q = lattice(n, N, 14)
    idx, tgt, valid = proposals(sites, n, bc == "periodic")
    f = O.FmmKmc(xyz, q, n, 3, 8, bc)
    cells = [0, 17, 63, 5, 40]
    before = [f.local(c) for c in cells]
    E0, K0, H0 = f.far()
    U0 = f.energy
    s = np.nonzero(valid)[0][3]
    i, t = idx[s], tgt[s]
    r = xyz[i].copy()
    d1 = f.accept(i, t)
    d2 = f.accept(i, r)
    after = [f.local(c) for c in cells]
    scale = max(np.max(np.abs(b)) for b in before)
    for b, a in zip(before, after):
        assert np.max(np.abs(a - b)) <= 1e-13 * scale
    assert f.energy == pytest.approx(U0 + d1 + d2, abs=1e-13)
    if bc == "free":
        assert d1 == pytest.approx(-d2, abs=1e-13)
    else:
        E1, K1, H1 = f.far()
        for x0, x1 in ((E0, E1), (K0, K1), (H0, H1)):
            assert np.max(np.abs(x1 - x0)) <= 1e-12 * max(1.0, np.max(np.abs(x0)))


def test_free_space_antisymmetry_after_accept():
    n, N = 16, 120
    sites, xyz, q = lattice(n, N, 15)
    idx, tgt, valid = proposals(sites, n, False)
    f = O.FmmKmc(xyz, q, n, 4, 10, "free")
    rng = np.random.default_rng(0)
    for s in rng.choice(np.nonzero(valid)[0], 5, replace=False):
        i, t = idx[s], tgt[s]
        r = f.positions()[i].copy()
        fwd = f.accept(i, t)
        back = f.propose([i], [r])[0]
        assert back == pytest.approx(-fwd, abs=1e-13 * max(1.0, abs(fwd)))


def test_lazy_and_full_agree_after_commits():
    n, N = 8, 60
    sites, xyz, q = lattice(n, N, 16)
    idx, tgt, valid = proposals(sites, n, True)
    full = O.FmmKmc(xyz, q, n, 3, 6, "periodic", lazy=False)
    lazy = O.FmmKmc(xyz, q, n, 3, 6, "periodic", lazy=True)
    vs = np.nonzero(valid)[0]
    for s in vs[[2, 30, 71]]:
        assert full.accept(idx[s], tgt[s]) == lazy.accept(idx[s], tgt[s])
    pos = full.positions()
    assert np.array_equal(pos, lazy.positions())
    sel = np.arange(0, len(idx), 7)
    a, b = full.propose(idx[sel], tgt[sel]), lazy.propose(idx[sel], tgt[sel])
    assert np.array_equal(np.isnan(a), np.isnan(b))
    m = ~np.isnan(a)
    assert np.max(np.abs(a[m] - b[m])) == 0.0


def test_far_field_K_tracks_root_multipole():
    n, N = 8, 40
    sites, xyz, q = lattice(n, N, 17)
    idx, tgt, valid = proposals(sites, n, True)
    f = O.FmmKmc(xyz, q, n, 3, 6, "periodic")
    for s in np.nonzero(valid)[0][[1, 9, 20, 33]]:
        f.accept(idx[s], tgt[s])
    E, K, H = f.far()
    root = f.rebuilt_multipole(1, 0)
    assert np.max(np.abs(K - root)) <= 1e-12 * np.max(np.abs(root))
    # E is the m -> -m partner of K
    for nn in range(7):
        for m in range(-nn, nn + 1):
            assert E[O.idx(nn, m)] == pytest.approx(K[O.idx(nn, -m)], abs=1e-12)


def test_masked_and_singular_proposals_are_nan():
    n, N = 8, 40
    sites, xyz, q = lattice(n, N, 18)
    f = O.FmmKmc(xyz, q, n, 3, 4, "free")
    d = f.propose([0, 0, 0, 1], [xyz[5], xyz[0], [n + 0.5, 1.5, 1.5], [0.5, 0.5, -0.5]])
    assert np.all(np.isnan(d))
