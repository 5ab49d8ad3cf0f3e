"""A uniform external field on free and periodic boxes (fmmkmc_set_field): every
proposal and accept adds -q E.d, d the hop (periodic: minimum image).  GPU
against O-fmm with the same field, through the C-ABI: lattice proposals (every
slot), generic proposals, 10 accepted moves and the energy, and a batch."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

E = np.array([0.25, -0.4, 0.6])


def guarded_err(d, ref):
    scale = float(np.mean(np.abs(ref)))
    return float(np.max(np.abs(d - ref) / np.maximum(np.abs(ref), scale)))


@pytest.mark.parametrize("bc,L,precision,tol", [("periodic", 4, "fp64", 1e-10), ("free", 4, "fp64", 1e-10),
                                                 ("periodic", 3, "mixed", 1e-5)])
def test_field_lattice_generic_and_accepts(bc, L, precision, tol):
    import torch
    from paper_1905_04065_amd import Context
    n, N, p = 16, 400, 8
    periodic = bc == "periodic"
    sites, xyz, q = W.lattice_charges(n, N, 1400 + L)
    ctx = Context(xyz, q, a=float(n), levels=L, order=p, bc=bc, precision=precision, lattice_n=n, device=0)
    U0 = ctx.initialise()
    ctx.set_field(E)
    ref = O.FmmKmc(xyz, q, n, L, p, bc, field=E)
    dU, mask = ctx.propose_lattice(W.HOPS26)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    t, v = O.lattice_targets(sites, n, W.HOPS26, periodic)
    v = v.reshape(-1)
    idx = np.repeat(np.arange(N), 26)
    e1 = guarded_err(dU[v], ref.propose(idx[v], W.site_xyz(t.reshape(-1)[v], n)))
    rng = np.random.default_rng(1401)
    gi = rng.integers(0, N, size=200)
    gt = xyz[gi] + rng.normal(scale=0.6, size=(200, 3))
    if not periodic:
        gt = np.clip(gt, 1e-3, n - 1e-3)
    e2 = guarded_err(ctx.propose_pairs(gi, gt).cpu().numpy(), ref.propose(gi, gt))
    u = W.commit_choices(10, 1402)
    cur = sites.copy()
    total = 0.0
    for k in range(10):
        t, vv = O.lattice_targets(cur, n, W.HOPS26, periodic)
        vs = np.nonzero(vv.reshape(-1))[0]
        s = vs[int(u[k] * len(vs))]
        i = int(s // 26)
        new = W.site_xyz([t.reshape(-1)[s]], n)[0]
        dg, dr = ctx.accept(i, new), ref.accept(i, new)
        assert abs(dg - dr) <= 1e-10 * max(abs(dr), 0.05)
        total += dg
        cur[i] = t.reshape(-1)[s]
    assert ctx.energy == pytest.approx(U0 + total, abs=1e-12 * max(1.0, abs(U0)))
    print(f"field {bc} L={L} {precision}: lattice {e1:.2e}, generic {e2:.2e}", flush=True)
    assert e1 < tol and e2 < tol
    ctx.close()


def test_field_batch_matches_single_context():
    from paper_1905_04065_amd import Batch, Context
    import torch
    Ns, ns, Ls = W.replica_sizes()
    ctxs, singles, reps = [], [], []
    for r in (203, 8):
        sites, xyz, q = W.replica_system(r, Ns[r], ns[r])
        for lst in (ctxs, singles):
            c = Context(xyz, q, a=float(ns[r]), levels=int(Ls[r]), order=6, bc="periodic", lattice_n=int(ns[r]),
                        device=0)
            c.initialise()
            c.set_field(E)
            lst.append(c)
        reps.append((int(ns[r]), sites.copy()))
    b = Batch(ctxs, W.HOPS6)
    u = np.random.default_rng(1403).random((4, 2))
    moved, site, dU = (x.cpu().numpy() for x in b.step(u))
    for r, (n, cur) in enumerate(reps):
        for s in range(4):
            d, m = singles[r].propose_lattice(W.HOPS6)
            torch.cuda.synchronize()
            vs = np.nonzero(m.cpu().numpy().reshape(-1))[0]
            slot = vs[int(u[s, r] * len(vs))]
            i = int(slot // 6)
            t, _ = O.lattice_targets(cur[i:i + 1], n, W.HOPS6[slot % 6:slot % 6 + 1], True)
            assert moved[s, r] == i and site[s, r] == int(t[0, 0])
            dd = singles[r].accept(i, W.site_xyz([int(t[0, 0])], n)[0])
            assert abs(dU[s, r] - dd) <= 1e-12 * max(abs(dd), 1e-3)
            cur[i] = int(t[0, 0])
    b.close()
