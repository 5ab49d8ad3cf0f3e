"""Batched replicas against the single-context path and the oracle.

Each replica of a batch is paired with an identical stand-alone context that
takes the same steps through the single-context API (lattice proposal pass,
the same dU-independent selection done on the host, accept).  The batched
kernels run the same per-block code, so moves must agree exactly and dU,
energies and the next proposal pass to rounding.  Two replicas are also
replayed by the oracle (O-fmm) and compared at the parity tolerance.  A second
batch takes the same steps as plain launches (profiling mode, no graph): the
graph replays must reproduce them.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [600, 1000, 2000, 3000, 1500, 4000]  # n_r = 11, 13, 16 (2x2x2 cells), 19, 15, 20


def replica(r, N, precision, p):
    n = int(math.ceil((2 * N) ** (1.0 / 3.0) - 1e-12))
    while n ** 3 < 2 * N:
        n += 1
    L = W.level_rule(N)
    sites, xyz, q = W.replica_system(r, N, n)
    return dict(n=n, N=N, L=L, p=p, sites=sites, xyz=xyz, q=q, precision=precision)


def make_ctx(rp):
    from paper_1905_04065_amd import Context
    ctx = Context(rp["xyz"], rp["q"], a=float(rp["n"]), levels=rp["L"], order=rp["p"], bc="periodic",
                  precision=rp["precision"], lattice_n=rp["n"], device=0)
    ctx.initialise()
    return ctx


def host_steps(ctx, rp, u, hops, cur):
    """the single-context path: proposal pass, selection, accept"""
    import torch
    K = len(hops)
    out = []
    last = None
    for s in range(len(u)):
        dU, mask = ctx.propose_lattice(hops)
        torch.cuda.synchronize()
        m = mask.cpu().numpy().reshape(-1).astype(bool)
        last = dU.cpu().numpy().reshape(-1)
        vs = np.nonzero(m)[0]
        if len(vs) == 0:
            out.append((-1, -1, float("nan")))
            continue
        slot = vs[int(u[s] * len(vs))]
        i = int(slot // K)
        t, _ = O.lattice_targets(cur[i:i + 1], rp["n"], hops[slot % K:slot % K + 1], True)
        new_site = int(t.reshape(-1)[0])
        d = ctx.accept(i, W.site_xyz([new_site], rp["n"])[0])
        cur[i] = new_site
        out.append((i, new_site, d))
    return out, last


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_context_and_oracle(precision):
    from paper_1905_04065_amd import Batch
    import torch
    p = 6
    hops = W.HOPS6
    reps = [replica(r, N, precision, p) for r, N in enumerate(SIZES)]
    print(f"batch of {len(reps)} replicas, n = {[rp['n'] for rp in reps]}, {precision}", flush=True)
    ctxs = [make_ctx(rp) for rp in reps]
    refs = [make_ctx(rp) for rp in reps]
    batch = Batch(ctxs, hops)
    R = len(reps)
    rng = np.random.default_rng(W.BASE_SEED + 50)
    steps1, steps2 = 12, 8
    u = rng.random((steps1 + steps2, R))
    moved, site, dU = batch.step(u[:steps1])
    info = batch.tune(rounds=3)
    print(f"  tuned: {info}", flush=True)
    moved2, site2, dU2 = batch.step(u[steps1:])
    moved = np.vstack([moved.cpu().numpy(), moved2.cpu().numpy()])
    site = np.vstack([site.cpu().numpy(), site2.cpu().numpy()])
    dU = np.vstack([dU.cpu().numpy(), dU2.cpu().numpy()])
    worst = 0.0
    curs = [rp["sites"].copy() for rp in reps]
    for r, rp in enumerate(reps):
        ref_steps, last = host_steps(refs[r], rp, u[:, r], hops, curs[r])
        for s, (i, ns, d) in enumerate(ref_steps):
            assert moved[s, r] == i and site[s, r] == ns, (r, s)
            worst = max(worst, abs(dU[s, r] - d) / max(abs(d), 1e-3))
        assert ctxs[r].energy == pytest.approx(refs[r].energy, rel=1e-12, abs=1e-12)
        np.testing.assert_array_equal(ctxs[r].positions().cpu().numpy(), refs[r].positions().cpu().numpy())
        bdU, bmask = batch.proposals(r)
        bdU = bdU.cpu().numpy().reshape(-1)
        v = bmask.cpu().numpy().reshape(-1).astype(bool)
        assert np.array_equal(np.isnan(bdU), ~v)
        assert np.max(np.abs(bdU[v] - last[v])) <= 1e-12 * max(1.0, float(np.max(np.abs(last[v]))))
    print(f"  {steps1 + steps2} steps x {R} replicas: moves identical, max dU difference {worst:.3e}", flush=True)
    assert worst <= 1e-12
    # the oracle replays two replicas' moves
    tol = 1e-10 if precision == "fp64" else 1e-5
    for r in (1, 2):
        rp = reps[r]
        ref = O.FmmKmc(rp["xyz"], rp["q"], float(rp["n"]), rp["L"], p, "periodic")
        scale = 0.0
        for s in range(steps1 + steps2):
            if moved[s, r] < 0:
                continue
            d_ref = ref.accept(int(moved[s, r]), W.site_xyz([site[s, r]], rp["n"])[0])
            scale = max(scale, abs(d_ref))
            assert abs(dU[s, r] - d_ref) <= 1e-10 * max(abs(d_ref), 0.05), (r, s, dU[s, r], d_ref)
        t, v = O.lattice_targets(curs[r], rp["n"], hops, True)
        v = v.reshape(-1)
        idx = np.repeat(np.arange(rp["N"]), len(hops))[v]
        d_ref = ref.propose(idx, W.site_xyz(t.reshape(-1)[v], rp["n"]))
        # the batch's last proposal pass preceded its last accept: compare a fresh pass
        dnow, mnow = ctxs[r].propose_lattice(hops)
        torch.cuda.synchronize()
        dnow = dnow.cpu().numpy().reshape(-1)
        assert np.array_equal(mnow.cpu().numpy().reshape(-1).astype(bool), v)
        err = float(np.max(np.abs(dnow[v] - d_ref) / np.maximum(np.abs(d_ref), np.mean(np.abs(d_ref)))))
        print(f"  replica {r} (n={rp['n']}{', 2x2x2 cells' if rp['n'] == 16 else ''}) vs O-fmm after "
              f"{steps1 + steps2} steps: {err:.3e}", flush=True)
        assert err < tol
    batch.close()


def test_graph_replays_match_plain_launches():
    """the same steps as one captured graph replayed, and as plain launches"""
    from paper_1905_04065_amd import Batch
    hops = W.HOPS6
    reps = [replica(r, N, "mixed", 6) for r, N in enumerate(SIZES[:4])]
    a = [make_ctx(rp) for rp in reps]
    b = [make_ctx(rp) for rp in reps]
    ba, bb = Batch(a, hops), Batch(b, hops)
    bb.set_profiling(True)
    u = np.random.default_rng(W.BASE_SEED + 51).random((10, len(reps)))
    for chunk in (u[:3], u[3:4], u[4:10]):  # several calls, eager work in between
        ma, sa, da = (x.cpu().numpy() for x in ba.step(chunk))
        mb, sb, db = (x.cpu().numpy() for x in bb.step(chunk))
        np.testing.assert_array_equal(ma, mb)
        np.testing.assert_array_equal(sa, sb)
        np.testing.assert_array_equal(da, db)
    t, n = bb.kernel_time("b_sweep")
    assert n == 10 * 1 and t > 0
    for x, y in zip(a, b):
        assert x.energy == y.energy
    ba.close()
    bb.close()


def test_single_context_accept_after_batched_steps():
    """after batched steps a context's own accept sees the moved charges"""
    from paper_1905_04065_amd import Batch
    hops = W.HOPS6
    rp = replica(0, 1000, "fp64", 6)
    c, ref = make_ctx(rp), make_ctx(rp)
    batch = Batch([c], hops)
    u = np.random.default_rng(W.BASE_SEED + 52).random((5, 1))
    moved, site, dU = (x.cpu().numpy() for x in batch.step(u))
    cur = rp["sites"].copy()
    for s in range(5):
        ref.accept(int(moved[s, 0]), W.site_xyz([site[s, 0]], rp["n"])[0])
        cur[int(moved[s, 0])] = site[s, 0]
    t, v = O.lattice_targets(cur, rp["n"], hops, True)
    vs = np.nonzero(v.reshape(-1))[0]
    slot = vs[len(vs) // 2]
    i, new = int(slot // 6), W.site_xyz([t.reshape(-1)[slot]], rp["n"])[0]
    d1 = c.accept(i, new)
    d2 = ref.accept(i, new)
    assert abs(d1 - d2) <= 1e-12 * max(1.0, abs(d2))
    assert c.energy == pytest.approx(ref.energy, rel=1e-12)
    batch.close()


@pytest.mark.parametrize("kind,precision", [(1, "fp64"), (2, "mixed")])
def test_propensity_weighted_selection(kind, precision):
    """Alg. 1 on the device: each step's move is the slot j with
    R_{j-1} < Q zeta <= R_j over the propensities of that step's proposal pass,
    and Delta t = -log(xi) / Q.  The reference sums the same dU (the batch's
    own proposals of the step) with numpy; the cumulative sums add in another
    order, so the chosen slot must hold T within rounding of its interval."""
    from paper_1905_04065_amd import Batch
    hops = W.HOPS6
    K = len(hops)
    nu, beta = 2.5, 1.7
    reps = [replica(r, N, precision, 6) for r, N in enumerate(SIZES[:4])]
    ctxs = [make_ctx(rp) for rp in reps]
    R = len(reps)
    batch = Batch(ctxs, hops)
    batch.set_rates(kind, nu, beta)
    rng = np.random.default_rng(W.BASE_SEED + 53)
    curs = [rp["sites"].copy() for rp in reps]
    n_steps = 10
    uu = rng.random((n_steps, R, 2))
    worst_t, worst_dt = 0.0, 0.0
    for s in range(n_steps):
        moved, site, dU, dt = (x.cpu().numpy() for x in batch.step(uu[s:s + 1], with_dt=True))
        for r, rp in enumerate(reps):
            pdU, pm = batch.proposals(r)  # the pass this step selected from
            pdU = pdU.cpu().numpy().reshape(-1)
            v = pm.cpu().numpy().reshape(-1).astype(bool)
            t, vv = O.lattice_targets(curs[r], rp["n"], hops, True)
            assert np.array_equal(v, vv.reshape(-1))
            rates = O.propensities(kind, nu, beta, pdU, v)
            cum = O.cumulative(rates)
            Q = cum[-1]
            T = Q * (1.0 - uu[s, r, 0])
            i = int(moved[0, r])
            assert i >= 0
            j = [slot for slot in range(i * K, i * K + K)
                 if v[slot] and t.reshape(-1)[slot] == site[0, r]]
            assert len(j) == 1, (s, r, i, site[0, r])
            j = j[0]
            lo, hi = (cum[j - 1] if j > 0 else 0.0), cum[j]
            slack = 1e-12 * Q
            assert lo - slack < T <= hi + slack, (s, r, j, lo, T, hi)
            worst_t = max(worst_t, max(lo - T, T - hi, 0.0) / Q)
            dt_ref = -math.log(1.0 - uu[s, r, 1]) / Q
            worst_dt = max(worst_dt, abs(dt[0, r] - dt_ref) / dt_ref)
            assert dt[0, r] == pytest.approx(dt_ref, rel=1e-12)
            # the accepted dU is the selected proposal's, recomputed in FP64 (relative
            # error on the scale of the pass's dU, as in the parity tests)
            tol = 1e-10 if precision == "fp64" else 1e-5
            assert abs(dU[0, r] - pdU[j]) <= tol * max(abs(pdU[j]), float(np.mean(np.abs(pdU[v]))))
            curs[r][i] = site[0, r]
    for r in range(R):
        np.testing.assert_allclose(ctxs[r].positions().cpu().numpy(), W.site_xyz(curs[r], reps[r]["n"]),
                                   rtol=0, atol=1e-12)
    print(f"  kind {kind}, {precision}: {n_steps} steps x {R} replicas, T outside its interval by "
          f"{worst_t:.2e} Q at most, dt within {worst_dt:.2e}", flush=True)
    batch.close()


def test_rates_at_zero_beta_are_a_uniform_choice():
    """beta = 0: every valid hop has propensity nu, so T = V nu zeta picks valid
    slot number ceil(V zeta) - 1 and Delta t = -log(xi) / (nu V) (closed form;
    the partial sums nu k are exact in FP64)"""
    from paper_1905_04065_amd import Batch
    hops = W.HOPS6
    K = len(hops)
    reps = [replica(r, N, "fp64", 6) for r, N in enumerate(SIZES[:3])]
    ctxs = [make_ctx(rp) for rp in reps]
    R = len(reps)
    batch = Batch(ctxs, hops)
    batch.set_rates(1, 3.0, 0.0)
    uu = np.random.default_rng(W.BASE_SEED + 54).random((4, R, 2))
    curs = [rp["sites"].copy() for rp in reps]
    for s in range(4):
        moved, site, dU, dt = (x.cpu().numpy() for x in batch.step(uu[s:s + 1], with_dt=True))
        for r, rp in enumerate(reps):
            t, v = O.lattice_targets(curs[r], rp["n"], hops, True)
            vs = np.nonzero(v.reshape(-1))[0]
            V = len(vs)
            T = (3.0 * V) * (1.0 - uu[s, r, 0])
            k = int(np.searchsorted(3.0 * np.arange(1, V + 1), T, side="left"))  # first R_k >= T
            slot = vs[k]
            assert moved[0, r] == slot // K and site[0, r] == t.reshape(-1)[slot], (s, r)
            assert dt[0, r] == pytest.approx(-math.log(1.0 - uu[s, r, 1]) / (3.0 * V), rel=1e-13)
            curs[r][slot // K] = site[0, r]
    # back to kind 0: one uniform per step, no time increment
    batch.set_rates(0)
    moved, site, dU, dt = (x.cpu().numpy() for x in batch.step(np.full((1, R), 0.5), with_dt=True))
    assert np.all(np.isnan(dt)) and np.all(moved >= 0)
    batch.close()


def test_set_rates_rejects_bad_arguments():
    from paper_1905_04065_amd import Batch, FmmKmcError
    rp = replica(0, 600, "fp64", 6)
    batch = Batch([make_ctx(rp)], W.HOPS6)
    for args in [(3, 1.0, 1.0), (-1, 1.0, 1.0), (1, 0.0, 1.0), (1, 1.0, -1.0), (2, float("inf"), 1.0),
                 (1, 1.0, float("nan"))]:
        with pytest.raises(FmmKmcError):
            batch.set_rates(*args)
    batch.close()


def test_replica_without_a_valid_hop_does_not_move():
    """degenerate case: a fully occupied lattice has no valid hop (Q = 0): the
    replica stays put (moved -1, dU NaN, Delta t +inf for rate kinds) while
    the other replica of the batch moves as usual"""
    from paper_1905_04065_amd import Batch, Context
    n = 8
    full_sites = np.arange(n ** 3)
    q_full = np.where(np.arange(n ** 3) % 2 == 0, 1.0, -1.0)
    np.random.default_rng(W.BASE_SEED + 55).shuffle(q_full)
    full = Context(W.site_xyz(full_sites, n), q_full, a=float(n), levels=3, order=4, bc="periodic",
                   lattice_n=n, device=0)
    full.initialise()
    rp = replica(1, 1000, "fp64", 4)
    rp["p"] = 4
    other = Context(rp["xyz"], rp["q"], a=float(rp["n"]), levels=rp["L"], order=4, bc="periodic",
                    lattice_n=rp["n"], device=0)
    other.initialise()
    U_full = full.energy
    batch = Batch([full, other], W.HOPS6)
    moved, site, dU = (x.cpu().numpy() for x in batch.step(np.full((3, 2), 0.3)))
    assert np.all(moved[:, 0] == -1) and np.all(site[:, 0] == -1) and np.all(np.isnan(dU[:, 0]))
    assert np.all(moved[:, 1] >= 0)
    bdU, bmask = batch.proposals(0)
    assert not bmask.cpu().numpy().any() and np.all(np.isnan(bdU.cpu().numpy()))
    batch.set_rates(1, 1.0, 1.0)
    moved, site, dU, dt = (x.cpu().numpy() for x in batch.step(np.full((2, 2, 2), 0.4), with_dt=True))
    assert np.all(moved[:, 0] == -1) and np.all(np.isinf(dt[:, 0])) and np.all(np.isfinite(dt[:, 1]))
    assert full.energy == U_full
    batch.close()


# replicas of the 256-replica workload (p = 10): the largest (n = 51, L = 5), two
# with 2 x 2 x 2 sites per fine cell (n = 32, L = 5 and n = 16, L = 4), the
# smallest (n = 13, L = 4) and four ordinary ones
CONFIG5_REPLICAS = [36, 4, 8, 203, 0, 1, 2, 3]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_config5_replicas_at_order_ten(precision, tol):
    """The batched kernels at the workload's own order and sizes: eight replicas
    drawn from the 256 (seeded as in the benchmark), six batched steps.  Moves
    exactly and dU to rounding against the single-context path; every accepted
    dU against O-fmm replaying the moves (FP64 accept path: 1e-10); then 256
    sampled slots of each replica's next proposal pass against O-fmm (formed
    lazily) at the precision's tolerance."""
    from paper_1905_04065_amd import Batch
    import torch
    p, hops, K = 10, W.HOPS6, 6
    Ns, ns, Ls = W.replica_sizes()
    reps = []
    for r in CONFIG5_REPLICAS:
        sites, xyz, q = W.replica_system(r, Ns[r], ns[r])
        reps.append(dict(n=int(ns[r]), N=int(Ns[r]), L=int(Ls[r]), p=p, sites=sites, xyz=xyz, q=q,
                         precision=precision))
    print(f"config-5 replicas {CONFIG5_REPLICAS}: n = {[rp['n'] for rp in reps]}, L = {[rp['L'] for rp in reps]}, "
          f"p = {p}, {precision}", flush=True)
    ctxs = [make_ctx(rp) for rp in reps]
    singles = [make_ctx(rp) for rp in reps]
    batch = Batch(ctxs, hops)
    batch.tune(rounds=2)
    R, steps = len(reps), 6
    u = np.random.default_rng(W.BASE_SEED + 57).random((steps, R))
    moved, site, dU = (x.cpu().numpy() for x in batch.step(u))
    worst_single, worst_acc, worst_slot = 0.0, 0.0, 0.0
    for r, rp in enumerate(reps):
        cur = rp["sites"].copy()
        ref_steps, _ = host_steps(singles[r], rp, u[:, r], hops, cur)
        for s, (i, ns_, d) in enumerate(ref_steps):
            assert moved[s, r] == i and site[s, r] == ns_, (r, s)
            worst_single = max(worst_single, abs(dU[s, r] - d) / max(abs(d), 1e-3))
        ref = O.FmmKmc(rp["xyz"], rp["q"], float(rp["n"]), rp["L"], p, "periodic", lazy=True)
        for s in range(steps):
            d_ref = ref.accept(int(moved[s, r]), W.site_xyz([site[s, r]], rp["n"])[0])
            worst_acc = max(worst_acc, abs(dU[s, r] - d_ref) / max(abs(d_ref), 0.05))
        dnow, mnow = ctxs[r].propose_lattice(hops)
        torch.cuda.synchronize()
        dnow = dnow.cpu().numpy().reshape(-1)
        t, v = O.lattice_targets(cur, rp["n"], hops, True)
        v = v.reshape(-1)
        assert np.array_equal(mnow.cpu().numpy().reshape(-1).astype(bool), v)
        pick = np.random.default_rng(W.BASE_SEED + 58 + r).choice(np.nonzero(v)[0], 256, replace=False)
        d_ref = ref.propose(pick // K, W.site_xyz(t.reshape(-1)[pick], rp["n"]))
        scale = float(np.mean(np.abs(dnow[v])))
        err = float(np.max(np.abs(dnow[pick] - d_ref) / np.maximum(np.abs(d_ref), scale)))
        worst_slot = max(worst_slot, err)
        print(f"  replica {CONFIG5_REPLICAS[r]} (n={rp['n']}, N={rp['N']}, L={rp['L']}): 256 sampled slots "
              f"{err:.3e}", flush=True)
        ref.close()
    print(f"  batched vs single-context dU {worst_single:.2e}; accepted dU vs O-fmm {worst_acc:.2e}; "
          f"sampled slots vs O-fmm {worst_slot:.2e}", flush=True)
    assert worst_single <= 1e-12
    assert worst_acc <= 1e-10
    assert worst_slot < tol
    batch.close()
