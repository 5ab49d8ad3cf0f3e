"""Invariants of the accept step on the GPU (Sec. 3 "Accept move", Sec. 3.1
"Accept move"), checked through the C-ABI.

* Multipoles on every level: after 25 accepted moves, Phi of every cell that a
  moved charge left or entered, on every level, equals the multipole of a fresh
  upward pass over the new positions (O-fmm), to rounding: the P2M update along
  the cell path is exact because M2M of a truncated multipole is exact.
* Round trip: a -> b -> a restores the energy, the positions, every dU of the
  next proposal pass and the multipoles, to rounding (free space and periodic).
* Free-space antisymmetry: after accepting a -> b, the proposal b -> a has
  dU = -dU(a -> b) to rounding (the moved charge never enters the local
  expansions of its own neighbourhood).
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def make_ctx(xyz, q, n, L, p, bc, precision="fp64"):
    from paper_1905_04065_amd import Context
    return Context(xyz, q, a=float(n), levels=L, order=p, bc=bc, precision=precision, lattice_n=n, device=0)


def to_library_storage(p, M):
    """the oracle's complex multipole (Greengard-Rokhlin normalisation) in the
    library's real storage: M_lib(n, m) = (-1)^m M(n, m) / sqrt((n-m)! (n+m)!)"""
    out = np.zeros((p + 1) ** 2)
    for n in range(p + 1):
        for m in range(n + 1):
            v = (-1) ** m * M[O.idx(n, m)] / math.sqrt(math.factorial(n - m) * math.factorial(n + m))
            if m == 0:
                out[n * n] = v.real
            else:
                out[n * n + 2 * m - 1] = v.real
                out[n * n + 2 * m] = v.imag
    return out


def moves(sites, n, count, seed, periodic):
    """seeded moves: half nearest-neighbour hops, half jumps to a random vacant site"""
    rng = np.random.default_rng(seed)
    cur = np.array(sites, np.int64).copy()
    occ = set(cur.tolist())
    out = []
    for s in range(count):
        while True:
            i = int(rng.integers(len(cur)))
            if s % 2 == 0:
                t, v = O.lattice_targets(cur[i:i + 1], n, W.HOPS6, periodic)
                k = int(rng.integers(6))
                new = int(t[0, k])
                if not v[0, k] or new in occ:  # off the lattice, or onto another charge
                    continue
            else:
                new = int(rng.integers(n ** 3))
                if new in occ:
                    continue
            break
        out.append((i, int(cur[i]), new))
        occ.discard(int(cur[i]))
        occ.add(new)
        cur[i] = new
    return out, cur


@pytest.mark.parametrize("bc", ["free", "periodic"])
def test_multipoles_on_every_level_follow_the_moves(bc):
    n, N, L, p = 16, 400, 4, 8
    periodic = bc == "periodic"
    sites, xyz, q = W.lattice_charges(n, N, 606)
    print(f"multipoles: n={n} N={N} L={L} p={p} {bc}, 25 moves", flush=True)
    ctx = make_ctx(xyz, q, n, L, p, bc)
    ctx.initialise()
    mv, cur = moves(sites, n, 25, 607, periodic)
    ref = O.FmmKmc(xyz, q, n, L, p, bc, lazy=True)
    touched = set()
    for i, old, new in mv:
        for s in (old, new):
            g = np.array([s // (n * n), (s // n) % n, s % n])
            for lev in range(1, L + 1):
                side = 2 ** (lev - 1)
                c = np.floor((g + 0.5) * side / n).astype(int)
                touched.add((lev, int((c[0] * side + c[1]) * side + c[2])))
        ctx.accept(i, W.site_xyz([new], n)[0])
        ref.accept(i, W.site_xyz([new], n)[0])
    worst, scale = 0.0, 0.0
    for lev, cell in sorted(touched):
        want = to_library_storage(p, ref.rebuilt_multipole(lev, cell))
        got = ctx.multipole(lev, cell)
        worst = max(worst, float(np.max(np.abs(got - want))))
        scale = max(scale, float(np.max(np.abs(want))))
    print(f"  {len(touched)} touched (level, cell) pairs: max |Phi - Phi_rebuilt| {worst:.3e} (scale {scale:.3e})",
          flush=True)
    assert worst <= 1e-12 * scale
    ctx.close()
    ref.close()


@pytest.mark.parametrize("bc,L", [("free", 4), ("periodic", 4), ("periodic", 3)])
def test_round_trip_restores_the_state(bc, L):
    import torch
    n, N, p = 16, 400, 8
    periodic = bc == "periodic"
    sites, xyz, q = W.lattice_charges(n, N, 608)
    print(f"round trip: n={n} N={N} L={L} p={p} {bc}", flush=True)
    ctx = make_ctx(xyz, q, n, L, p, bc)
    U0 = ctx.initialise()
    d0, m0 = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    d0, m0 = d0.cpu().numpy(), m0.cpu().numpy()
    phi0 = [ctx.multipole(lev, c) for lev in range(1, L + 1) for c in range(0, 8 ** (lev - 1), 7)]
    # a long move and a hop, each undone
    mv, _ = moves(sites, n, 2, 609, periodic)
    worst_anti = 0.0
    total = 0.0
    for k, (i, old, new) in enumerate(mv):
        fwd = ctx.accept(i, W.site_xyz([new], n)[0])
        # free space, a hop inside the 27 cells around the charge: the return
        # move undoes the energy change exactly (the charge never enters a local
        # expansion of its own neighbourhood); after a long move the two dU's
        # differ at truncation level (tree versus P2L update of the far cells)
        hop = k == 0
        if hop and not periodic:
            back = float(ctx.propose_pairs([i], [W.site_xyz([old], n)[0]]).cpu().numpy()[0])
            worst_anti = max(worst_anti, abs(back + fwd) / max(abs(fwd), 1e-3))
        bwd = ctx.accept(i, W.site_xyz([old], n)[0])
        total += fwd + bwd
        if hop and not periodic:
            assert abs(fwd + bwd) <= 1e-12 * max(1.0, abs(fwd))
    d1, m1 = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    d1, m1 = d1.cpu().numpy(), m1.cpu().numpy()
    np.testing.assert_array_equal(m1, m0)
    v = m0.astype(bool)
    err = float(np.max(np.abs(d1[v] - d0[v])) / np.mean(np.abs(d0[v])))
    np.testing.assert_array_equal(ctx.positions().cpu().numpy(), xyz)
    phi1 = [ctx.multipole(lev, c) for lev in range(1, L + 1) for c in range(0, 8 ** (lev - 1), 7)]
    perr = max(float(np.max(np.abs(a - b))) for a, b in zip(phi0, phi1))
    pscale = max(float(np.max(np.abs(a))) for a in phi0)
    print(f"  every dU restored to {err:.2e} of the mean; multipoles to {perr / pscale:.2e}; energy "
          f"{ctx.energy - U0 - total:.2e}; antisymmetry {worst_anti:.2e}", flush=True)
    assert err <= 1e-12
    assert perr <= 1e-13 * pscale
    # the energy is the initial one plus the accepted dU's; in periodic boxes the
    # two dU's cancel only to truncation level (the copies' P2L updates)
    assert abs(ctx.energy - (U0 + total)) <= 1e-12 * max(1.0, abs(U0))
    if not periodic:
        assert worst_anti <= 1e-12
    ctx.close()


def test_free_space_antisymmetry_for_neighbour_hops():
    """after a -> b, dU(b -> a) = -dU(a -> b) for 20 seeded hops"""
    n, N, L, p = 16, 300, 4, 8
    sites, xyz, q = W.lattice_charges(n, N, 610)
    ctx = make_ctx(xyz, q, n, L, p, "free")
    ctx.initialise()
    rng = np.random.default_rng(611)
    cur = sites.copy()
    worst = 0.0
    for _ in range(20):
        t, v = O.lattice_targets(cur, n, W.HOPS6, False)
        vs = np.nonzero(v.reshape(-1))[0]
        s = int(vs[rng.integers(len(vs))])
        i = s // 6
        old = W.site_xyz([cur[i]], n)[0]
        fwd = ctx.accept(i, W.site_xyz([t.reshape(-1)[s]], n)[0])
        back = float(ctx.propose_pairs([i], [old]).cpu().numpy()[0])
        worst = max(worst, abs(back + fwd) / max(abs(fwd), 1e-3))
        cur[i] = t.reshape(-1)[s]
    print(f"free-space antisymmetry over 20 hops: {worst:.2e}", flush=True)
    assert worst <= 1e-12
    ctx.close()
