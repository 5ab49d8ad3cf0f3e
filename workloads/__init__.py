"""Seeded synthetic inputs for the FMM-KMC hot path.

This module only draws inputs: lattice sites, charges, hop offsets, replica
sizes and the sequence of moves to commit.  It holds none of the method's
arithmetic, so both the GPU library's callers and the CPU oracle can be fed
from it without sharing any computation.

Lattice convention: an n x n x n simple cubic lattice of spacing h, sites at
((i + 1/2) h, (j + 1/2) h, (k + 1/2) h), box [0, a)^3 with a = n h.  Sites are
numbered s = (i * n + j) * n + k.
"""
import math

import numpy as np

BASE_SEED = 190504065

#: the six nearest-neighbour hops, in the order +x, -x, +y, -y, +z, -z
HOPS6 = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.int32)
#: first, second and third shells: {-1,0,1}^3 without 0, lexicographic
HOPS26 = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
                   if (i, j, k) != (0, 0, 0)], np.int32)
#: 6 face and 8 body-diagonal hops (the strong/weak scaling setup of Sec. 6.3)
HOPS14 = np.concatenate([HOPS6, np.array([[i, j, k] for i in (-1, 1) for j in (-1, 1) for k in (-1, 1)],
                                         np.int32)])


def level_rule(N):
    """Levels L (root = 1) for N charges: L = 1 + max(3, floor(log8(N/2))), in integers."""
    k, v = 0, 8
    while v <= N // 2:
        k += 1
        v *= 8
    return 1 + max(3, k)


def lattice_charges(n, N, seed, h=1.0):
    """N distinct sites drawn uniformly from n^3, half +1 and half -1 (shuffled).

    Returns (sites int64[N], xyz float64[N,3], q float64[N]).
    """
    if N > n ** 3:
        raise ValueError("more charges than sites")
    rng = np.random.default_rng(seed)
    sites = rng.choice(n ** 3, size=N, replace=False).astype(np.int64)
    q = np.ones(N)
    q[N // 2:] = -1.0
    if N % 2:
        q[-1] = 1.0
    rng.shuffle(q)
    return sites, site_xyz(sites, n, h), q


def site_xyz(sites, n, h=1.0):
    sites = np.asarray(sites, np.int64)
    i = sites // (n * n)
    j = (sites // n) % n
    k = sites % n
    return (np.stack([i, j, k], 1).astype(np.float64) + 0.5) * h


CONFIGS = {
    1: dict(bc="free", n=32, N=1000, L=4, p=8, hops="6", precision="fp64"),
    2: dict(bc="periodic", n=64, N=100000, L=6, p=12, hops="6", precision="fp64", steps=100),
    3: dict(bc="free", n=32, N=1000, L=4, p=8, hops="6", precision="mixed", commits=10000),
    4: dict(bc="periodic", n=128, N=1000000, L=7, p=12, hops="26", precision="both"),
    5: dict(bc="periodic", replicas=256, Nmin=1000, Nmax=65536, p=10, hops="6", precision="mixed"),
}


def hops(name):
    return {"6": HOPS6, "14": HOPS14, "26": HOPS26}[str(name)]


def config_system(cid, h=1.0):
    """(sites, xyz, q, params) of configs 1-4, seeded with BASE_SEED + cid."""
    c = dict(CONFIGS[cid])
    sites, xyz, q = lattice_charges(c["n"], c["N"], BASE_SEED + cid, h)
    c["a"] = c["n"] * h
    c["h"] = h
    return sites, xyz, q, c


def replica_sizes(count=256, Nmin=1000, Nmax=65536, seed=BASE_SEED + 5):
    """N_r: the even integer nearest exp(U(ln Nmin, ln Nmax)); lattice side
    n_r = ceil((2 N_r)^(1/3)) (about 50 % occupancy); levels by level_rule."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(Nmin), math.log(Nmax), size=count)
    N = (2 * np.rint(np.exp(u) / 2)).astype(np.int64)
    n = np.array([int(math.ceil((2 * v) ** (1.0 / 3.0) - 1e-12)) for v in N], np.int64)
    for r in range(count):
        while n[r] ** 3 < 2 * N[r]:
            n[r] += 1
    L = np.array([level_rule(int(v)) for v in N], np.int64)
    return N, n, L


def replica_system(r, N, n, h=1.0):
    return lattice_charges(int(n), int(N), BASE_SEED * 1000 + r, h)


def commit_choices(count, seed):
    """Uniform numbers u in [0, 1) for a move selection that does not depend
    on dU: the move taken is valid slot floor(u * n_valid) in slot order."""
    rng = np.random.default_rng(seed)
    return rng.random(count)


def perturbed_lattice(N, density, seed, jitter=0.1):
    """The error-study setup of Sec. 6.1: N charges (N a cube) on a cubic
    lattice at the given number density with small random perturbations,
    alternating signs shuffled.  Returns (xyz, q, a)."""
    m = int(round(N ** (1.0 / 3.0)))
    if m ** 3 != N:
        raise ValueError("N must be a cube")
    a = (N / density) ** (1.0 / 3.0)
    s = a / m
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    xyz = (g + 0.5 + rng.uniform(-jitter, jitter, size=g.shape)) * s
    q = np.ones(N)
    q[N // 2:] = -1.0
    rng.shuffle(q)
    return xyz, q, a
