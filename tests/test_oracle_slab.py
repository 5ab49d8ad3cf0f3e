"""Pins of the slab oracle (grounded plates by the first mirror image, Sec. 2.2.2).

* The doubled system's potential vanishes on both plates (the Dirichlet
  condition the construction is for), checked with O-exact Ewald sums; a
  mid-slab point is not at zero potential, so the check is not vacuous.
* The pair-move formula (two single moves plus the partner bracket) equals the
  difference of two full Ewald energies of the doubled system.
* A charge and its mirror have equal single-move dU (mirror symmetry).
* The field term is exactly -E_z q dz.
* O-fmm slab proposals agree with the O-exact slab to the truncation level.
"""
import numpy as np
import pytest

import oracle as O
from oracle import slab as S


def system(seed, n=8, N=6):
    rng = np.random.default_rng(seed)
    half = n // 2
    sites = rng.choice(n * n * half, N, replace=False)
    ijk = np.stack([sites // (n * half), (sites // half) % n, sites % half], 1)
    xyz = (ijk + 0.5).astype(np.float64)
    q = np.where(rng.random(N) < 0.5, 1.0, -1.0)
    return float(n), xyz, q


def potential_difference(xyz2, q2, a, p0, p1):
    """phi(p1) - phi(p0) of the doubled system: dU of a unit test charge"""
    allx = np.vstack([xyz2, p0])
    allq = np.concatenate([q2, [1.0]])
    return O.ewald_dU(allx, allq, a, [len(q2)], [p1])[0]


def test_plates_are_at_zero_potential():
    a, xyz, q = system(1)
    xyz2, q2 = S.mirror_system(xyz, q, a)
    rng = np.random.default_rng(2)
    p0 = np.array([0.3, 1.7, 0.0])
    worst = 0.0
    for _ in range(4):
        for zp in (0.0, a / 2):
            p1 = np.array([rng.random() * a, rng.random() * a, zp])
            worst = max(worst, abs(potential_difference(xyz2, q2, a, p0, p1)))
    assert worst < 1e-12
    mid = potential_difference(xyz2, q2, a, p0, np.array([2.1, 3.3, a / 4]))
    assert abs(mid) > 1e-3


def test_pair_formula_equals_energy_difference():
    a, xyz, q = system(3)
    N = len(q)
    xyz2, q2 = S.mirror_system(xyz, q, a)
    E0 = O.ewald_energy(xyz2, q2, a)
    done = 0
    for i, hop in [(0, (0, 0, 1)), (1, (0, 0, -1)), (2, (1, 0, 0)), (3, (0, 1, 1)), (4, (0, -1, -1)),
                   (5, (-1, 0, 1))]:
        t = xyz[i] + np.array(hop, float)
        t[:2] %= a
        if not (0 < t[2] < a / 2) or any(np.allclose(t, x) for x in xyz):
            continue
        tm = S.mirror_point(t, a)
        after = xyz2.copy()
        after[i], after[N + i] = t, tm
        full = O.ewald_energy(after, q2, a) - E0
        du_i = O.ewald_dU(xyz2, q2, a, [i], [t])[0]
        du_m = O.ewald_dU(xyz2, q2, a, [N + i], [tm])[0]
        X = q[i] * (-q[i]) * S.pair_bracket(xyz2[i], xyz2[N + i], t, tm, a)
        assert abs(du_i - du_m) <= 1e-12 * max(1.0, abs(du_i))
        assert abs(du_i + du_m + X - full) <= 1e-11 * max(1.0, abs(full))
        done += 1
    assert done >= 3


def test_field_term_and_fmm_slab_against_exact():
    a, xyz, q = system(5, n=16, N=24)
    N = len(q)
    ez = 0.37
    o0 = S.SlabOracle(xyz, q, a, 4, 10, ez=0.0)
    o1 = S.SlabOracle(xyz, q, a, 4, 10, ez=ez)
    xyz2, q2 = S.mirror_system(xyz, q, a)
    worst, done = 0.0, 0
    for i in range(0, N, 3):
        for hop in [(1, 0, 0), (0, 0, 1), (0, 0, -1)]:
            t = xyz[i] + np.array(hop, float)
            t[:2] %= a
            if not (0 < t[2] < a / 2) or any(np.allclose(t, x) for x in xyz):
                continue
            d0, d1 = o0.propose(i, t), o1.propose(i, t)
            assert d1 - d0 == pytest.approx(-ez * q[i] * hop[2], abs=1e-13)
            tm = S.mirror_point(t, a)
            ex = 0.5 * (O.ewald_dU(xyz2, q2, a, [i], [t])[0] + O.ewald_dU(xyz2, q2, a, [N + i], [tm])[0]
                        - q[i] ** 2 * S.pair_bracket(xyz2[i], xyz2[N + i], t, tm, a))
            worst = max(worst, abs(d0 - ex) / max(abs(ex), 0.05))
            done += 1
    assert done >= 10
    assert worst < 1e-3  # truncation at p = 10, L = 4
