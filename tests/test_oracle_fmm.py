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
    t, valid = O.lattice_targets(sites, n, hops, periodic)
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


# ---- pins of the accept step's fine-level sweep (Sec. 3 "Accept move", Sec. 3.1 "Accept move") ----

def _long_moves(f, sites, n, L, count, seed, min_cells=3):
    """accept `count` seeded moves of random charges to random vacant sites at
    least `min_cells` fine cells away (long moves cross many cells, so every
    fine cell's expansion sees a moved copy leave or arrive outside its near
    field); returns the current lattice sites"""
    rng = np.random.default_rng(seed)
    cur = np.array(sites, np.int64).copy()
    occ = set(cur.tolist())
    w = n / 2 ** (L - 1)
    N = len(cur)
    for _ in range(count):
        while True:
            i = int(rng.integers(N))
            s = int(rng.integers(n ** 3))
            if s in occ:
                continue
            a = W.site_xyz([cur[i]], n)[0]
            b = W.site_xyz([s], n)[0]
            if np.max(np.abs(np.floor(a / w) - np.floor(b / w))) >= min_cells:
                break
        f.accept(i, b)
        occ.discard(int(cur[i]))
        occ.add(s)
        cur[i] = s
    return cur


def test_accept_sweep_long_moves_keep_free_space_dU_exact():
    """After six long accepted moves, O-fmm's dU of every hop of every charge
    matches the direct pair sum of the new configuration (O-exact) as closely as
    a fresh system does (p = 16: truncation ~1e-7 of the mean).  Catches a sweep
    that does nothing (the moved charge stays at its old place in every far
    cell's expansion: errors ~1e-2), one that adds with the wrong sign, and one
    that updates the wrong cells (a near cell counted twice or a far cell
    missed)."""
    n, N, L, p = 16, 150, 4, 16
    sites, xyz, q = lattice(n, N, 21)
    f = O.FmmKmc(xyz, q, n, L, p, "free")
    idx, tgt, valid = proposals(sites, n, False)
    ref0 = O.direct_dU(xyz, q, idx[valid], tgt[valid])
    e0 = np.max(np.abs(f.propose(idx[valid], tgt[valid]) - ref0)) / np.mean(np.abs(ref0))
    cur = _long_moves(f, sites, n, L, 6, 5)
    xyz1 = W.site_xyz(cur, n)
    np.testing.assert_array_equal(f.positions(), xyz1)
    idx, tgt, valid = proposals(cur, n, False)
    ref1 = O.direct_dU(xyz1, q, idx[valid], tgt[valid])
    e1 = np.max(np.abs(f.propose(idx[valid], tgt[valid]) - ref1)) / np.mean(np.abs(ref1))
    assert e0 < 2e-7
    assert e1 < 3 * e0 + 1e-9, (e0, e1)
    # and the total energy follows the accepted dU's to the direct energy
    assert abs(f.energy - O.direct_energy(xyz1, q)) < 1e-6 * abs(O.direct_energy(xyz1, q))


def test_accept_sweep_long_moves_keep_periodic_dU_exact():
    """The periodic sweep moves all 27 copies of V_box: after five long moves
    O-fmm's dU matches tin-foil Ewald for the new configuration within the
    pre-commit band (p = 18).  Catches a sweep that moves only the primary copy
    (missing images: the 26 copies around the box stay behind), a sign error,
    or a wrong near test for wrapped copies."""
    n, N, L, p = 8, 40, 3, 18
    sites, xyz, q = lattice(n, N, 22)
    f = O.FmmKmc(xyz, q, n, L, p, "periodic")
    cur = _long_moves(f, sites, n, L, 5, 6, min_cells=2)
    xyz1 = W.site_xyz(cur, n)
    idx, tgt, valid = proposals(cur, n, True)
    ref = O.ewald_dU(xyz1, q, n, idx[valid], tgt[valid])
    d = f.propose(idx[valid], tgt[valid])
    err = np.max(np.abs(d - ref)) / np.mean(np.abs(ref))
    assert err < 2e-6, err
    assert f.energy == pytest.approx(O.ewald_energy(xyz1, q, n), abs=1e-6)


def _copies_outside_near(pos, g_cell, n_fine, w, a, periodic):
    """the copies pos + a nu (nu in V_box, or nu = 0 in free space) whose fine
    cell (extended coordinates) is not one of the 27 cells around g_cell"""
    out = []
    rng = (-1, 0, 1) if periodic else (0,)
    for i in rng:
        for j in rng:
            for k in rng:
                y = np.array(pos, float) + a * np.array([i, j, k], float)
                gy = np.floor(y / w).astype(int)
                if np.max(np.abs(gy - np.asarray(g_cell))) > 1:
                    out.append(y)
    return out


@pytest.mark.parametrize("bc,n,N,L,p", [("free", 16, 120, 4, 14), ("periodic", 8, 40, 3, 14)])
def test_accept_changes_each_local_expansion_by_its_far_copies(bc, n, N, L, p):
    """One accepted move, every fine cell beta: at the cell centre a local
    expansion reduces to its constant term, so the change of Psi_beta there must
    equal, to rounding, the Coulomb change sum q (1/|c - r' - a nu| - 1/|c - r -
    a nu|) over exactly the copies outside the 27 cells around beta (free
    space: nu = 0 only), and at an interior point the same sum within the
    truncation bound.  Catches a no-op sweep, a flipped sign, missing periodic
    copies and a wrong near test (a near copy added, a far copy skipped)."""
    periodic = bc == "periodic"
    sites, xyz, q = lattice(n, N, 23)
    f = O.FmmKmc(xyz, q, n, L, p, bc)
    nf = 2 ** (L - 1)
    w = n / nf
    # a move between two cells that are not neighbours
    i = 0
    r = xyz[i].copy()
    occ = set(sites.tolist())
    rng = np.random.default_rng(7)
    while True:
        s = int(rng.integers(n ** 3))
        t = W.site_xyz([s], n)[0]
        if s not in occ and np.max(np.abs(np.floor(t / w) - np.floor(r / w))) >= 2:
            break
    cells = range(nf ** 3)
    before = [f.local(c) for c in cells]
    f.accept(i, t)
    off = np.array([0.3, -0.2, 0.25]) * w
    worst_c, worst_x, scale = 0.0, 0.0, 0.0
    changed = 0
    for c in cells:
        g = np.array([c // (nf * nf), (c // nf) % nf, c % nf])
        ctr = (g + 0.5) * w
        dL = f.local(c) - before[c]
        want_c = sum(q[i] / np.linalg.norm(ctr - y) for y in _copies_outside_near(t, g, nf, w, n, periodic)) - \
            sum(q[i] / np.linalg.norm(ctr - y) for y in _copies_outside_near(r, g, nf, w, n, periodic))
        x = ctr + off
        want_x = sum(q[i] / np.linalg.norm(x - y) for y in _copies_outside_near(t, g, nf, w, n, periodic)) - \
            sum(q[i] / np.linalg.norm(x - y) for y in _copies_outside_near(r, g, nf, w, n, periodic))
        got_c = O.eval_local(p, dL, ctr, ctr)
        got_x = O.eval_local(p, dL, ctr, x)
        worst_c = max(worst_c, abs(got_c - want_c))
        worst_x = max(worst_x, abs(got_x - want_x))
        scale = max(scale, abs(want_c))
        changed += abs(want_c) > 1e-12
    assert changed > nf ** 3 // 2  # most cells see the move
    assert worst_c <= 1e-13 * scale, (worst_c, scale)
    # interior point at |x - c| = 0.45 w, copies beyond 1.5 w: ratio 0.3, bound ~ 0.3^(p+1) / w
    assert worst_x <= 2 * 0.3 ** (p + 1) / w * 10, (worst_x, scale)


def test_exact_self_image_matches_ewald(periodic_box):
    """With the exact self-image term (q^2 (psi_self - psi(r' - r)) in place of the
    V_box self sum, the constant and 1/2 dE.R'dK) O-fmm still converges to tin-foil
    Ewald: within the same band as the paper's terms at p = 18, and the two forms
    differ only at truncation level (they approximate the same quantity)."""
    n, xyz, q, idx, tgt, valid, ref, Ue = periodic_box
    lit = O.FmmKmc(xyz, q, n, 3, 18, "periodic").propose(idx[valid], tgt[valid])
    ex = O.FmmKmc(xyz, q, n, 3, 18, "periodic", self_image="exact").propose(idx[valid], tgt[valid])
    scale = np.mean(np.abs(ref[valid]))
    assert np.max(np.abs(ex - ref[valid])) < 2e-6 * scale
    assert np.max(np.abs(ex - lit)) < 2e-6 * scale
    errs = []
    for p in (6, 10, 14):
        d = O.FmmKmc(xyz, q, n, 3, p, "periodic", self_image="exact").propose(idx[valid], tgt[valid])
        errs.append(np.max(np.abs(d - ref[valid])))
    assert errs[0] > 5 * errs[1] > 25 * errs[2]


def test_exact_self_image_accepts_and_round_trips():
    """the exact self-image term in the accept step: the round trip restores the
    expansions and the accepted dU's match Ewald energy differences"""
    n, N = 8, 40
    sites, xyz, q = lattice(n, N, 24)
    idx, tgt, valid = proposals(sites, n, True)
    f = O.FmmKmc(xyz, q, n, 3, 18, "periodic", self_image="exact")
    s = np.nonzero(valid)[0][5]
    i, t = idx[s], tgt[s]
    d1 = f.accept(i, t)
    xyz1 = xyz.copy()
    xyz1[i] = t
    assert d1 == pytest.approx(O.ewald_energy(xyz1, q, n) - O.ewald_energy(xyz, q, n), abs=2e-6)
    d2 = f.accept(i, xyz[i])
    assert d2 == pytest.approx(-d1, abs=2e-6)


# ---- per-level expansions (the survey's next step f1; Introduction and Sec. 7) ----

@pytest.mark.parametrize("bc,L", [("free", 4), ("periodic", 3), ("periodic", 4)])
def test_per_level_expansions_equal_accumulated_before_commits(bc, L):
    """Summing every level's own expansion at a point equals the accumulated
    fine-level expansion to rounding (L2L of a truncated local expansion is an
    exact polynomial translation), so before any commit the two modes agree"""
    n, N, p = 16, 300, 8
    sites, xyz, q = lattice(n, N, 25)
    idx, tgt, valid = proposals(sites, n, bc == "periodic")
    a = O.FmmKmc(xyz, q, n, L, p, bc).propose(idx[valid], tgt[valid])
    f = O.FmmKmc(xyz, q, n, L, p, bc, per_level=True)
    b = f.propose(idx[valid], tgt[valid])
    assert np.max(np.abs(a - b)) <= 1e-12 * np.mean(np.abs(a))
    assert f.energy == pytest.approx(O.FmmKmc(xyz, q, n, L, p, bc).energy, rel=1e-13)


@pytest.mark.parametrize("bc,n,N,L,p", [("free", 16, 150, 4, 16), ("periodic", 8, 40, 3, 18)])
def test_per_level_commits_keep_dU_exact(bc, n, N, L, p):
    """After long moves the per-level update keeps O-fmm's dU as close to
    O-exact (direct sum, tin-foil Ewald) as before the commits (high p).
    Catches a per-level rule that misses copies (a wrong interaction-list
    test, missing images) or updates with the wrong sign."""
    periodic = bc == "periodic"
    sites, xyz, q = lattice(n, N, 26)
    f = O.FmmKmc(xyz, q, n, L, p, bc, per_level=True)
    cur = _long_moves(f, sites, n, L, 6 if not periodic else 5, 8, min_cells=3 if not periodic else 2)
    xyz1 = W.site_xyz(cur, n)
    idx, tgt, valid = proposals(cur, n, periodic)
    ref = O.ewald_dU(xyz1, q, n, idx[valid], tgt[valid]) if periodic else O.direct_dU(xyz1, q, idx[valid],
                                                                                        tgt[valid])
    d = f.propose(idx[valid], tgt[valid])
    err = np.max(np.abs(d - ref)) / np.mean(np.abs(ref))
    assert err < (2e-6 if periodic else 3e-7), err


@pytest.mark.parametrize("bc,n,N,L,p", [("free", 16, 120, 4, 10), ("periodic", 8, 40, 3, 10),
                                        ("periodic", 16, 120, 4, 10)])
def test_per_level_accept_changes_each_cell_by_its_interaction_list(bc, n, N, L, p):
    """One accepted move, every cell of every level: at a cell's centre its
    expansion reduces to the constant term, so the change of Psi_{l,beta} there
    must equal, to rounding, the Coulomb change of exactly the copies whose
    level-l cell is in the interaction list of beta (outside the 27 cells
    around beta, inside the children of the 27 around its parent)"""
    periodic = bc == "periodic"
    sites, xyz, q = lattice(n, N, 27)
    f = O.FmmKmc(xyz, q, n, L, p, bc, per_level=True)
    start = 2 if periodic else 3
    i = 1
    r = xyz[i].copy()
    occ = set(sites.tolist())
    rng = np.random.default_rng(9)
    while True:
        s = int(rng.integers(n ** 3))
        if s not in occ:
            t = W.site_xyz([s], n)[0]
            break
    levels = range(start, L + 1)
    before = {(l, c): f.level_local(l, c) for l in levels for c in range(8 ** (l - 1))}
    f.accept(i, t)
    rngc = (-1, 0, 1) if periodic else (0,)
    worst, scale = 0.0, 0.0
    for (l, c), b0 in before.items():
        side = 2 ** (l - 1)
        w = n / side
        g = np.array([c // (side * side), (c // side) % side, c % side])
        ctr = (g + 0.5) * w
        want = 0.0
        for pos, sgn in ((t, 1.0), (r, -1.0)):
            for nu in [(a, b, cc) for a in rngc for b in rngc for cc in rngc]:
                y = pos + n * np.array(nu, float)
                G = np.floor(y / w).astype(int)
                near = np.max(np.abs(G - g)) <= 1
                parent_near = np.max(np.abs(np.floor_divide(G, 2) - g // 2)) <= 1
                if not near and parent_near:
                    want += sgn * q[i] / np.linalg.norm(ctr - y)
        got = O.eval_local(p, f.level_local(l, c) - b0, ctr, ctr)
        worst = max(worst, abs(got - want))
        scale = max(scale, abs(want))
    assert scale > 0
    assert worst <= 1e-13 * scale, (worst, scale)


def test_per_level_round_trip_restores_state():
    n, N, L, p = 16, 120, 4, 8
    sites, xyz, q = lattice(n, N, 28)
    f = O.FmmKmc(xyz, q, n, L, p, "periodic", per_level=True)
    cells = [(2, 3), (3, 17), (4, 100), (4, 511)]
    before = [f.level_local(l, c) for l, c in cells]
    idx, tgt, valid = proposals(sites, n, True)
    s = np.nonzero(valid)[0][7]
    f.accept(idx[s], tgt[s])
    f.accept(idx[s], xyz[idx[s]])
    for (l, c), b in zip(cells, before):
        assert np.max(np.abs(f.level_local(l, c) - b)) <= 1e-13 * np.max(np.abs(b))


@pytest.mark.parametrize("bc", ["free", "periodic"])
def test_uniform_field_adds_the_work_over_the_hop(bc):
    """A uniform field E adds -q E.d to every proposal (d the hop; across a
    periodic face the minimum image), exactly, and the energy of accepted moves
    follows; the field term does not change the electrostatic part"""
    n, N = 8, 40
    sites, xyz, q = lattice(n, N, 29)
    idx, tgt, valid = proposals(sites, n, bc == "periodic", W.HOPS26)
    E = np.array([0.3, -0.2, 0.7])
    f0 = O.FmmKmc(xyz, q, n, 3, 8, bc)
    f1 = O.FmmKmc(xyz, q, n, 3, 8, bc, field=E)
    d0 = f0.propose(idx[valid], tgt[valid])
    d1 = f1.propose(idx[valid], tgt[valid])
    disp = tgt[valid] - xyz[idx[valid]]
    disp -= n * np.round(disp / n)  # the hop itself (the targets of wrapped hops lie across the box)
    assert np.all(np.abs(disp) <= 1.0)
    np.testing.assert_allclose(d1 - d0, -q[idx[valid]] * (disp @ E), rtol=0, atol=1e-13)
    s = np.nonzero(valid)[0][3]
    a0, a1 = f0.accept(idx[s], tgt[s]), f1.accept(idx[s], tgt[s])
    assert a1 - a0 == pytest.approx(-q[idx[s]] * float((tgt[s] - xyz[idx[s]] - n * np.round((tgt[s] - xyz[idx[s]]) / n)) @ E),
                                    abs=1e-13)
