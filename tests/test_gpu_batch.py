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
        t, _ = W.lattice_targets(cur[i:i + 1], rp["n"], hops[slot % K:slot % K + 1], True)
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
        t, v = W.lattice_targets(curs[r], rp["n"], hops, True)
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
    t, v = W.lattice_targets(cur, rp["n"], hops, True)
    vs = np.nonzero(v.reshape(-1))[0]
    slot = vs[len(vs) // 2]
    i, new = int(slot // 6), W.site_xyz([t.reshape(-1)[slot]], rp["n"])[0]
    d1 = c.accept(i, new)
    d2 = ref.accept(i, new)
    assert abs(d1 - d2) <= 1e-12 * max(1.0, abs(d2))
    assert c.energy == pytest.approx(ref.energy, rel=1e-12)
    batch.close()
