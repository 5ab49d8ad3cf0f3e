"""Per-level local expansions (fmmkmc_params.per_level = 1) on the GPU against
O-fmm with the same mode: each level keeps its own interaction-list terms,
proposals sum the levels, and an accept updates per level only the cells
whose interaction list holds the moved charge.  Same tolerances as the other
parity tests (guarded relative error 1e-10 FP64, 1e-5 mixed; masks and
positions exact)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def guarded_err(d, ref, scale=None):
    if scale is None:
        scale = max(float(np.mean(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(d - ref) / np.maximum(np.abs(ref), scale)))


def make_ctx(xyz, q, a, L, p, bc, precision="fp64", lattice_n=0, self_image="expansion"):
    from paper_1905_04065_amd import Context
    return Context(xyz, q, a=float(a), levels=L, order=p, bc=bc, precision=precision, lattice_n=lattice_n,
                   device=0, per_level=True, self_image=self_image)


def slots(sites, n, hops, periodic):
    t, v = O.lattice_targets(sites, n, hops, periodic)
    return np.repeat(np.arange(len(sites)), len(hops)), W.site_xyz(t.reshape(-1), n), v.reshape(-1)


def moves(sites, n, count, seed, periodic):
    """seeded moves, alternately a neighbour hop and a jump to a random vacant site"""
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
        out.append((i, new))
        occ.discard(int(cur[i]))
        occ.add(new)
        cur[i] = new
    return out, cur


CASES = [
    # (n, N, L, p, bc, hops, precision, tol)
    (16, 400, 4, 8, "periodic", "26", "fp64", 1e-10),   # 2x2x2 sites per cell: coarse levels by orbits
    (16, 300, 3, 8, "periodic", "6", "fp64", 1e-10),    # general lattice, one coarse level
    (20, 500, 4, 7, "periodic", "6", "fp64", 1e-10),    # non-integer cell width
    (16, 300, 4, 8, "free", "6", "fp64", 1e-10),        # free space, 2x2x2
    (16, 200, 3, 6, "free", "6", "fp64", 1e-10),        # free space with no coarse level
    (32, 3000, 5, 8, "periodic", "6", "fp64", 1e-10),   # three coarse levels by orbits
    (16, 800, 4, 8, "periodic", "26", "mixed", 1e-5),
]


@pytest.mark.parametrize("n,N,L,p,bc,hops,precision,tol", CASES)
def test_per_level_lattice_commits_every_slot(n, N, L, p, bc, hops, precision, tol):
    """every slot before any accept, 20 accepted moves (hops and long jumps)
    against O-fmm replaying them, then every slot again"""
    import torch
    periodic = bc == "periodic"
    H = W.hops(hops)
    sites, xyz, q = W.lattice_charges(n, N, 1300 + n + L)
    print(f"per-level: n={n} N={N} L={L} p={p} {bc} {len(H)} hops {precision}", flush=True)
    ctx = make_ctx(xyz, q, n, L, p, bc, precision, lattice_n=n)
    U = ctx.initialise()
    ref = O.FmmKmc(xyz, q, n, L, p, bc, per_level=True)
    assert abs(U - ref.energy) <= 1e-11 * max(1.0, abs(ref.energy))
    errs = []
    for phase in range(2):
        dU, mask = ctx.propose_lattice(H)
        torch.cuda.synchronize()
        dU = dU.cpu().numpy().reshape(-1)
        cur = np.floor(ctx.positions().cpu().numpy()).astype(np.int64) @ np.array([n * n, n, 1])
        idx, tgt, v = slots(cur, n, H, periodic)
        assert np.array_equal(mask.cpu().numpy().reshape(-1).astype(bool), v)
        assert np.all(np.isnan(dU[~v]))
        errs.append(guarded_err(dU[v], ref.propose(idx[v], tgt[v])))
        if phase == 0:
            mv, _ = moves(cur, n, 20, 1301 + L, periodic)
            worst = 0.0
            for i, new in mv:
                pos = W.site_xyz([new], n)[0]
                d_gpu, d_ref = ctx.accept(i, pos), ref.accept(i, pos)
                worst = max(worst, abs(d_gpu - d_ref) / max(abs(d_ref), 0.05))
            np.testing.assert_array_equal(ctx.positions().cpu().numpy(), ref.positions())
    print(f"  every slot {errs[0]:.3e}; 20 accepts {worst:.3e}; every slot after {errs[1]:.3e}", flush=True)
    assert worst <= 1e-10
    assert max(errs) < tol
    assert ctx.energy == pytest.approx(ref.energy, abs=1e-10 * max(1.0, abs(ref.energy)))
    ctx.close()


@pytest.mark.parametrize("bc", ["free", "periodic"])
def test_per_level_generic_and_potential(bc):
    """off-lattice generic proposals and potentials after accepts"""
    rng = np.random.default_rng(1310)
    a, N, L, p = 12.0, 240, 4, 7
    xyz = rng.uniform(0, a, size=(N, 3))
    q = np.array([1.0, -1.0] * (N // 2))
    ctx = make_ctx(xyz, q, a, L, p, bc)
    ctx.initialise()
    ref = O.FmmKmc(xyz, q, a, L, p, bc, per_level=True)
    for _ in range(6):
        i = int(rng.integers(N))
        new = rng.uniform(0.01, a - 0.01, size=3)
        d_gpu, d_ref = ctx.accept(i, new), ref.accept(i, new)
        assert abs(d_gpu - d_ref) <= 1e-10 * max(abs(d_ref), 0.05)
    idx = rng.integers(0, N, size=300)
    tgt = np.clip(ctx.positions().cpu().numpy()[idx] + rng.normal(scale=0.7, size=(300, 3)), 1e-3, a - 1e-3)
    err = guarded_err(ctx.propose_pairs(idx, tgt).cpu().numpy(), ref.propose(idx, tgt))
    pts = rng.uniform(0, a, size=(40, 3))
    got = ctx.potential(pts).cpu().numpy()
    want = np.array([ref.potential(x) for x in pts])
    perr = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    print(f"per-level generic {bc}: proposals {err:.2e}, potentials {perr:.2e}", flush=True)
    assert err < 1e-10 and perr < 1e-11
    ctx.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_per_level_batch_config5_replicas(precision, tol):
    """batched per-level replicas (p = 10): moves exactly and dU to rounding
    against the single-context path, two replicas against O-fmm"""
    from paper_1905_04065_amd import Batch
    import torch
    p, hops, K = 10, W.HOPS6, 6
    Ns, ns, Ls = W.replica_sizes()
    pick = [36, 4, 203, 0]
    reps = []
    for r in pick:
        sites, xyz, q = W.replica_system(r, Ns[r], ns[r])
        reps.append(dict(n=int(ns[r]), N=int(Ns[r]), L=int(Ls[r]), sites=sites, xyz=xyz, q=q))

    def mk(rp):
        c = make_ctx(rp["xyz"], rp["q"], rp["n"], rp["L"], p, "periodic", precision, lattice_n=rp["n"])
        c.initialise()
        return c
    ctxs = [mk(rp) for rp in reps]
    singles = [mk(rp) for rp in reps]
    batch = Batch(ctxs, hops)
    steps = 5
    u = np.random.default_rng(W.BASE_SEED + 60).random((steps, len(reps)))
    moved, site, dU = (x.cpu().numpy() for x in batch.step(u))
    worst = 0.0
    for r, rp in enumerate(reps):
        cur = rp["sites"].copy()
        for s in range(steps):
            d, m = singles[r].propose_lattice(hops)
            torch.cuda.synchronize()
            vs = np.nonzero(m.cpu().numpy().reshape(-1))[0]
            slot = vs[int(u[s, r] * len(vs))]
            i = int(slot // K)
            t, _ = O.lattice_targets(cur[i:i + 1], rp["n"], hops[slot % K:slot % K + 1], True)
            assert moved[s, r] == i and site[s, r] == int(t[0, 0]), (r, s)
            dd = singles[r].accept(i, W.site_xyz([int(t[0, 0])], rp["n"])[0])
            worst = max(worst, abs(dU[s, r] - dd) / max(abs(dd), 1e-3))
            cur[i] = int(t[0, 0])
        rp["cur"] = cur
    assert worst <= 1e-12
    for r in (0, 1):
        rp = reps[r]
        ref = O.FmmKmc(rp["xyz"], rp["q"], float(rp["n"]), rp["L"], p, "periodic", lazy=True, per_level=True)
        for s in range(steps):
            d_ref = ref.accept(int(moved[s, r]), W.site_xyz([site[s, r]], rp["n"])[0])
            assert abs(dU[s, r] - d_ref) <= 1e-10 * max(abs(d_ref), 0.05)
        dnow, mnow = ctxs[r].propose_lattice(hops)
        torch.cuda.synchronize()
        dnow = dnow.cpu().numpy().reshape(-1)
        idx, tgt, v = slots(rp["cur"], rp["n"], hops, True)
        assert np.array_equal(mnow.cpu().numpy().reshape(-1).astype(bool), v)
        pk = np.random.default_rng(W.BASE_SEED + 61 + r).choice(np.nonzero(v)[0], 256, replace=False)
        err = guarded_err(dnow[pk], ref.propose(idx[pk], tgt[pk]), float(np.mean(np.abs(dnow[v]))))
        print(f"per-level batch {precision}: replica {pick[r]} (n={rp['n']}, L={rp['L']}) 256 slots {err:.2e}; "
              f"batched vs single {worst:.2e}", flush=True)
        assert err < tol
        ref.close()
    batch.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_per_level_config4(precision, tol):
    """config 4 (128^3, N = 1e6, 26 hops, L = 7, p = 12): 3 accepted moves
    against O-fmm (formed lazily, same mode), then 256 sampled slots"""
    import torch
    sites, xyz, q, c = W.config_system(4)
    hops = W.hops(c["hops"])
    K = len(hops)
    print(f"config 4 per-level {precision}", flush=True)
    ctx = make_ctx(xyz, q, c["a"], c["L"], c["p"], "periodic", precision, lattice_n=c["n"])
    ctx.initialise()
    ref = O.FmmKmc(xyz, q, c["a"], c["L"], c["p"], "periodic", lazy=True, per_level=True)
    mv, cur = moves(sites, c["n"], 3, 1320, True)
    for i, new in mv:
        pos = W.site_xyz([new], c["n"])[0]
        d_gpu, d_ref = ctx.accept(i, pos), ref.accept(i, pos)
        assert abs(d_gpu - d_ref) <= 1e-10 * max(abs(d_ref), 0.05), (d_gpu, d_ref)
    dU, mask = ctx.propose_lattice(hops)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    idx, tgt, v = slots(cur, c["n"], hops, True)
    assert np.array_equal(mask.cpu().numpy().reshape(-1).astype(bool), v)
    pk = np.random.default_rng(W.BASE_SEED + 43).choice(np.nonzero(v)[0], 256, replace=False)
    err = guarded_err(dU[pk], ref.propose(idx[pk], tgt[pk]), float(np.mean(np.abs(dU[v]))))
    print(f"  after 3 accepts, 256 sampled slots: {err:.3e}", flush=True)
    assert err < tol
    ctx.close()
    ref.close()
