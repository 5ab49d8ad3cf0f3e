"""The allocation-free proposal entry point (fmmkmc_propose_noalloc) against
fmmkmc_propose on the same inputs, through the C-ABI: two calls in a row, the
second smaller than the first, in a periodic and a free-space box; the same
kernels run on the same inputs, so the outputs must agree bit for bit (NaN in
the same slots).  Oversized calls and malformed CSR arrays are refused before
any computation."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _case(bc, seed):
    import torch
    from paper_1905_04065_amd import Context
    n, N, L, p = 16, 400, 4, 8
    sites, xyz, q = W.lattice_charges(n, N, seed)
    ctx = Context(xyz, q, a=float(n), levels=L, order=p, bc=bc, lattice_n=0, device=0)
    ctx.initialise()
    return ctx, xyz, n, N, torch


def _groups(rng, N, xyz, n, G, per, free):
    idx = rng.integers(0, N, size=G)
    counts = rng.integers(1, 2 * per, size=G)
    offs = np.concatenate([[0], np.cumsum(counts)])
    S = int(offs[-1])
    tgt = xyz[np.repeat(idx, counts)] + rng.normal(scale=0.8, size=(S, 3))
    if free:
        tgt = np.clip(tgt, 1e-3, n - 1e-3)
    return idx, offs, tgt


@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_noalloc_matches_propose_on_two_calls(bc):
    ctx, xyz, n, N, torch = _case(bc, 700 + (bc == "free"))
    rng = np.random.default_rng(701)
    for G, per in ((900, 6), (150, 3)):  # about 5400 targets, then about 450
        idx, offs, tgt = _groups(rng, N, xyz, n, G, per, bc == "free")
        S = int(offs[-1])
        print(f"{bc}: {G} groups, {S} targets", flush=True)
        ref = ctx.propose(idx, offs, tgt, check=False)[0].cpu().numpy()
        d_idx = torch.as_tensor(idx, dtype=torch.int64, device="cuda")
        d_offs = torch.as_tensor(offs, dtype=torch.int64, device="cuda")
        d_tgt = torch.as_tensor(tgt, dtype=torch.float64, device="cuda").contiguous()
        d_out = torch.full((S,), 7.0, dtype=torch.float64, device="cuda")
        rc = ctx.propose_noalloc(d_idx, d_offs, d_tgt, d_out, check=False)
        got = d_out.cpu().numpy()
        assert rc in (0, 3)  # ECOINCIDENT only if a random target hit a charge exactly
        np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
        np.testing.assert_array_equal(got[~np.isnan(ref)], ref[~np.isnan(ref)])
    ctx.close()


def test_noalloc_refuses_oversized_and_malformed_calls():
    from paper_1905_04065_amd import EINVAL
    ctx, xyz, n, N, torch = _case("periodic", 702)
    idx = torch.zeros(1, dtype=torch.int64, device="cuda")
    big = torch.tensor([0, (1 << 18) + 1], dtype=torch.int64, device="cuda")
    tgt = torch.zeros(3, dtype=torch.float64, device="cuda")
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    assert ctx.propose_noalloc(idx, big, tgt, out, check=False) == EINVAL
    bad = torch.tensor([1, 2], dtype=torch.int64, device="cuda")  # offs[0] != 0
    assert ctx.propose_noalloc(idx, bad, tgt, out, check=False) == EINVAL
    far = torch.tensor([N + 5], dtype=torch.int64, device="cuda")
    one = torch.tensor([0, 1], dtype=torch.int64, device="cuda")
    assert ctx.propose_noalloc(far, one, tgt, out, check=False) == EINVAL
    assert float(out.cpu()[0]) == 7.0  # nothing written
    # and a valid call afterwards still works
    t1 = torch.as_tensor(xyz[3] + 0.5, dtype=torch.float64, device="cuda").contiguous()
    assert ctx.propose_noalloc(idx, one, t1, out, check=False) == 0
    ref = ctx.propose(idx, one, t1).cpu().numpy()
    assert float(out.cpu()[0]) == ref[0]
    ctx.close()
