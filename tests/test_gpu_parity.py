"""GPU parity: the HIP library against the CPU oracle O-fmm (same L, p, box, BC).

Tolerance (FP64): |dU - dU*| <= 1e-10 max(|dU*|, <|dU*|>) for every valid slot,
the guarded relative error of the dU target with the mean magnitude as the
floor (dU is a difference of potentials ~10-100 times larger, so FP64 rounding
alone leaves ~1e-14 of the mean).  Mixed precision: the same form with 1e-5.
Masked slots must be NaN on both sides and identical masks (integer work:
exact).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def guarded_err(d, ref):
    scale = max(float(np.mean(np.abs(ref))), 1e-300)
    return float(np.max(np.abs(d - ref) / np.maximum(np.abs(ref), scale)))


def lattice_case(n, N, seed, periodic, hops=W.HOPS6):
    sites, xyz, q = W.lattice_charges(n, N, seed)
    t, valid = O.lattice_targets(sites, n, hops, periodic)
    idx = np.repeat(np.arange(N), len(hops))
    tgt = W.site_xyz(t.reshape(-1), n)
    return sites, xyz, q, idx, tgt, valid.reshape(-1)


def make_ctx(xyz, q, n, L, p, bc, precision="fp64", lattice=True):
    from paper_1905_04065_amd import Context
    return Context(xyz, q, a=float(n), levels=L, order=p, bc=bc, precision=precision,
                   lattice_n=n if lattice else 0, device=0)


CASES = [
    # (n, N, L, p, bc)   geometry of the site kernel
    (12, 60, 2, 6, "free"),        # no interaction lists: direct sums only
    (16, 200, 3, 6, "free"),       # 4 sites per cell axis: general site kernel
    (16, 300, 4, 8, "free"),       # 2 sites per cell axis: the 2x2x2 kernel
    (16, 300, 3, 8, "periodic"),   # general site kernel, periodic
    (16, 400, 4, 8, "periodic"),   # 2x2x2 kernel, periodic
    (20, 500, 4, 7, "periodic"),   # non-integer cell width (2.5 sites), ties at cell faces
    (13, 300, 4, 6, "periodic"),   # 1.625 sites per cell edge: cells of one and of two planes
    (6, 40, 4, 5, "periodic"),     # 0.75 sites per cell edge: cells with no plane at all
    (10, 100, 4, 6, "free"),       # 1.25 sites per cell edge, clamped boxes at the faces
    (16, 200, 2, 6, "free"),       # 8 sites per cell axis: boxes beyond the 1/sqrt table (computed 1/|d|)
]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_general_lattice_staged_in_chunks(precision, tol):
    """A general lattice (3.75 sites per cell edge: cells of 3 or 4 planes,
    near-field boxes up to 12 planes) whose blocks' union boxes exceed the LDS
    tile, so the site kernel stages them in several x-plane chunks and reads
    the longest fixed-length rows.  The whole mask bit-exactly, a seeded
    sample of slots against O-fmm (formed lazily)."""
    import torch
    n, L, p = 60, 5, 8
    N = 2 * (int(0.4 * n ** 3) // 2)
    sites, xyz, q = W.lattice_charges(n, N, 2024)
    t, v = O.lattice_targets(sites, n, W.HOPS6, True)
    v = v.reshape(-1)
    K = len(W.HOPS6)
    print(f"general lattice n={n} N={N} L={L} p={p} periodic {precision}", flush=True)
    ctx = make_ctx(xyz, q, n, L, p, "periodic", precision)
    ctx.initialise()
    dU, mask = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    assert np.array_equal(mask.cpu().numpy().reshape(-1).astype(bool), v)
    assert np.all(np.isnan(dU[~v])) and not np.any(np.isnan(dU[v]))
    ref = O.FmmKmc(xyz, q, n, L, p, "periodic", lazy=True)
    pick = np.random.default_rng(W.BASE_SEED + 60).choice(np.nonzero(v)[0], 256, replace=False)
    d_ref = ref.propose(pick // K, W.site_xyz(t.reshape(-1)[pick], n))
    scale = float(np.mean(np.abs(dU[v])))
    err = float(np.max(np.abs(dU[pick] - d_ref) / np.maximum(np.abs(d_ref), scale)))
    print(f"  256 sampled slots of {v.sum()}: max guarded rel err {err:.3e}", flush=True)
    assert err < tol
    ctx.close()
    ref.close()


@pytest.mark.parametrize("n,N,L,p,bc", CASES)
def test_lattice_proposals_match_oracle(n, N, L, p, bc):
    import torch
    periodic = bc == "periodic"
    sites, xyz, q, idx, tgt, valid = lattice_case(n, N, 1000 + n + L, periodic)
    print(f"case n={n} N={N} L={L} p={p} {bc}", flush=True)
    ctx = make_ctx(xyz, q, n, L, p, bc)
    U = ctx.initialise()
    dU, mask = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    mask = mask.cpu().numpy().reshape(-1).astype(bool)
    assert np.array_equal(mask, valid)
    assert np.all(np.isnan(dU[~valid]))
    ref = O.FmmKmc(xyz, q, n, L, p, bc)
    d_ref = ref.propose(idx[valid], tgt[valid])
    err = guarded_err(dU[valid], d_ref)
    print(f"  max guarded rel err {err:.3e}; U {U:.15g} vs {ref.energy:.15g}", flush=True)
    assert err < 1e-10
    assert abs(U - ref.energy) <= 1e-11 * max(1.0, abs(ref.energy))
    ctx.close()


@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_general_lattice_charges_not_exact_in_fp32(bc):
    """FP64 on a general lattice (2.5 sites per cell edge) with charges +-0.3,
    which FP32 rounds: the site kernel cannot stage them in FP32 and takes its
    box-row body for every block.  Every valid slot against O-fmm."""
    import torch
    periodic = bc == "periodic"
    n, N, L, p = 20, 500, 4, 7
    sites, xyz, q, idx, tgt, valid = lattice_case(n, N, 4242, periodic)
    q = 0.3 * q
    print(f"charges +-0.3: n={n} N={N} L={L} p={p} {bc}", flush=True)
    ctx = make_ctx(xyz, q, n, L, p, bc)
    ctx.initialise()
    dU, mask = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    assert np.array_equal(mask.cpu().numpy().reshape(-1).astype(bool), valid)
    d_ref = O.FmmKmc(xyz, q, n, L, p, bc).propose(idx[valid], tgt[valid])
    err = guarded_err(dU[valid], d_ref)
    print(f"  max guarded rel err {err:.3e}", flush=True)
    assert err < 1e-10
    ctx.close()


@pytest.mark.parametrize("bc,L", [("free", 3), ("periodic", 3)])
def test_generic_proposals_match_oracle(bc, L):
    """propose(P) with arbitrary (off-lattice) targets."""
    import torch
    rng = np.random.default_rng(7)
    a, N, p = 10.0, 120, 7
    xyz = rng.uniform(0, a, size=(N, 3))
    q = np.array([1.0, -1.0] * (N // 2))
    ctx = make_ctx(xyz, q, a, L, p, bc, lattice=False)
    ctx.initialise()
    idx = rng.integers(0, N, size=300)
    tgt = xyz[idx] + rng.normal(scale=0.6, size=(300, 3))
    if bc == "free":
        tgt = np.clip(tgt, 1e-6, a - 1e-6)
    d = ctx.propose_pairs(idx, tgt).cpu().numpy()
    ref = O.FmmKmc(xyz, q, a, L, p, bc).propose(idx, tgt)
    err = guarded_err(d, ref)
    print(f"generic {bc}: max guarded rel err {err:.3e}", flush=True)
    assert err < 1e-10
    ctx.close()


def test_potential_matches_oracle():
    rng = np.random.default_rng(8)
    n, N, L, p = 16, 300, 4, 8
    sites, xyz, q, *_ = lattice_case(n, N, 77, True)
    ctx = make_ctx(xyz, q, n, L, p, "periodic")
    ctx.initialise()
    pts = rng.uniform(0, n, size=(50, 3))
    ex = rng.integers(-1, N, size=50)
    pts[ex >= 0] = xyz[ex[ex >= 0]]
    got = ctx.potential(pts, ex).cpu().numpy()
    ref = O.FmmKmc(xyz, q, n, L, p, "periodic")
    want = np.array([ref.potential(pts[j], ex[j]) for j in range(50)])
    assert np.max(np.abs(got - want)) < 1e-11 * np.max(np.abs(want))
    ctx.close()


@pytest.mark.parametrize("n,N,L,p,bc", [(16, 300, 4, 8, "free"), (16, 400, 4, 8, "periodic"),
                                        (16, 300, 3, 6, "periodic")])
def test_commits_match_oracle_replay(n, N, L, p, bc):
    """accept a seeded, dU-independent sequence of moves on both sides, then
    compare every proposal; the accepted dU's and the energy are compared too."""
    import torch
    periodic = bc == "periodic"
    sites, xyz, q, idx, tgt, valid = lattice_case(n, N, 4242 + L, periodic)
    ctx = make_ctx(xyz, q, n, L, p, bc)
    ctx.initialise()
    ref = O.FmmKmc(xyz, q, n, L, p, bc)
    u = W.commit_choices(25, 99)
    cur_sites = sites.copy()
    for step in range(25):
        t, vmask = O.lattice_targets(cur_sites, n, W.HOPS6, periodic)
        vs = np.nonzero(vmask.reshape(-1))[0]
        s = vs[int(u[step] * len(vs))]
        i, k = divmod(int(s), 6)
        newpos = W.site_xyz([t.reshape(-1)[s]], n)[0]
        d_gpu = ctx.accept(i, newpos)
        d_ref = ref.accept(i, newpos)
        assert abs(d_gpu - d_ref) <= 1e-10 * max(abs(d_ref), 0.05), (step, d_gpu, d_ref)
        cur_sites[i] = t.reshape(-1)[s]
    assert ctx.energy == pytest.approx(ref.energy, abs=1e-10 * abs(ref.energy))
    np.testing.assert_array_equal(ctx.positions().cpu().numpy(), ref.positions())
    t, vmask = O.lattice_targets(cur_sites, n, W.HOPS6, periodic)
    dU, mask = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    m = vmask.reshape(-1)
    assert np.array_equal(mask.cpu().numpy().reshape(-1).astype(bool), m)
    idx2 = np.repeat(np.arange(N), 6)
    d_ref = ref.propose(idx2[m], W.site_xyz(t.reshape(-1)[m], n))
    err = guarded_err(dU[m], d_ref)
    print(f"after commits {bc} L={L}: max guarded rel err {err:.3e}", flush=True)
    assert err < 1e-10
    ctx.close()


def test_mixed_precision_free_space():
    """config-3 shape at reduced N: FP32 fine-level evaluation, FP64 everywhere else"""
    import torch
    n, N, L, p = 32, 1000, 4, 8
    sites, xyz, q, idx, tgt, valid = lattice_case(n, N, W.BASE_SEED + 3, False)
    ctx = make_ctx(xyz, q, n, L, p, "free", precision="mixed")
    ctx.initialise()
    dU, mask = ctx.propose_lattice(W.HOPS6)
    torch.cuda.synchronize()
    dU = dU.cpu().numpy().reshape(-1)
    ref = O.FmmKmc(xyz, q, n, L, p, "free").propose(idx[valid], tgt[valid])
    err = guarded_err(dU[valid], ref)
    print(f"mixed free: max guarded rel err {err:.3e}", flush=True)
    assert err < 1e-5
    ctx.close()


def test_mixed_precision_periodic_s2():
    import torch
    n, N, L, p = 16, 800, 4, 8
    sites, xyz, q, idx, tgt, valid = lattice_case(n, N, 31337, True)
    ctx = make_ctx(xyz, q, n, L, p, "periodic", precision="mixed")
    ctx.initialise()
    dU, mask = ctx.propose_lattice(W.HOPS26)
    torch.cuda.synchronize()
    sites_, xyz_, q_, idx26, tgt26, valid26 = lattice_case(n, N, 31337, True, W.HOPS26)
    dU = dU.cpu().numpy().reshape(-1)
    ref = O.FmmKmc(xyz, q, n, L, p, "periodic").propose(idx26[valid26], tgt26[valid26])
    err = guarded_err(dU[valid26], ref)
    print(f"mixed periodic s2 26 hops: max guarded rel err {err:.3e}", flush=True)
    assert err < 1e-5
    ctx.close()


def test_propose_with_dats():
    """App. C: types with c_t hops, masks; forbidden / beyond-c_t entries are NaN."""
    import torch
    n, N, L, p = 16, 200, 4, 6
    sites, xyz, q, idx, tgt, valid = lattice_case(n, N, 555, True)
    K = 4
    Ct = [0, 2, 3, 4]
    rng = np.random.default_rng(3)
    T = rng.integers(0, 4, size=N).astype(np.int32)
    R = np.zeros((N, K, 3))
    M = np.ones((N, K), np.uint8)
    t6, v6 = O.lattice_targets(sites, n, W.HOPS6, True)
    for i in range(N):
        for k in range(K):
            R[i, k] = W.site_xyz([t6[i, k]], n)[0]
            M[i, k] = 1 if v6[i, k] else 0
    ctx = make_ctx(xyz, q, n, L, p, "periodic")
    ctx.initialise()
    U = ctx.propose_dats(K, Ct, T, R.reshape(N, 3 * K), M).cpu().numpy()
    ref = O.FmmKmc(xyz, q, n, L, p, "periodic")
    use = (np.arange(K)[None, :] < np.array(Ct)[T][:, None]) & (M == 1)
    ii, kk = np.nonzero(use)
    d_ref = ref.propose(ii, R[ii, kk])
    assert np.all(np.isnan(U[~use]))
    assert guarded_err(U[ii, kk], d_ref) < 1e-10
    ctx.close()


def test_error_codes():
    from paper_1905_04065_amd import FmmKmcError, EDOMAIN, ECOINCIDENT, EINVAL
    n, N = 8, 40
    sites, xyz, q, *_ = lattice_case(n, N, 5, False)
    with pytest.raises(FmmKmcError) as e:
        make_ctx(np.vstack([xyz, xyz[:1]]), np.append(q, 1.0), n, 3, 4, "free")
    assert e.value.code == ECOINCIDENT
    with pytest.raises(FmmKmcError) as e:
        make_ctx(xyz + 0.25, q, n, 3, 4, "free")  # off the lattice
    assert e.value.code == EDOMAIN
    ctx = make_ctx(xyz, q, n, 3, 4, "free")
    ctx.initialise()
    with pytest.raises(FmmKmcError) as e:
        ctx.accept(0, xyz[1])
    assert e.value.code == ECOINCIDENT
    with pytest.raises(FmmKmcError) as e:
        ctx.accept(0, [n + 0.5, 0.5, 0.5])
    assert e.value.code == EDOMAIN
    with pytest.raises(FmmKmcError) as e:
        ctx.accept(N, xyz[0])
    assert e.value.code == EINVAL
    d, rc = ctx.propose_pairs([0, 1], [xyz[2], [0.5, 0.5, n + 3.0]], check=False)
    assert rc == EDOMAIN
    assert np.all(np.isnan(d.cpu().numpy()))
    ctx.close()
