"""KMC bookkeeping of the oracle: lattice proposal sets and Alg. 1's selection.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): plain numpy statements of
what the library computes on the device around the electrostatics.

* ``lattice_targets``: the proposal set of App. C on a site lattice.  Every
  charge proposes a hop to the site at each lattice offset; in a periodic box
  the target wraps into the box (Sec. 6.3 runs periodic lattices), in free
  space a target off the lattice is masked (a charge cannot leave the box).
  A target on an occupied site is masked too (its energy change is undefined,
  App. C).
* ``propensities`` / ``select_slot`` / ``time_increment``: Alg. 1 of Sec. 2.1.
  Each proposal j gets a rate r_j (the rate function of Sec. 6: nu exp(-beta
  dU), or its Metropolis form nu min(1, exp(-beta dU)); masked slots 0); with
  cumulative sums R_j and total Q, the event taken is the j with
  R_{j-1} < Q zeta <= R_j, and time advances by -log(xi) / Q.

Pinned in tests/test_oracle_kmc.py against brute force on positions (targets),
hand-summed intervals and the beta = 0 closed form (selection).
"""
import numpy as np


def lattice_targets(sites, n, offsets, periodic):
    """Target site of every (charge, hop) slot and its validity.

    sites: lattice index s = (i n + j) n + k of each charge; offsets: K x 3
    integer hops.  Returns (tsite int64[N, K], valid bool[N, K]); a masked slot
    of a free-space hop off the lattice carries the clamped site index."""
    sites = np.asarray(sites, np.int64)
    ijk = np.stack([sites // (n * n), (sites // n) % n, sites % n], 1)[:, None, :] + \
        np.asarray(offsets, np.int64)[None, :, :]
    if periodic:
        inside = np.ones(ijk.shape[:2], bool)
        ijk = np.mod(ijk, n)
    else:
        inside = np.all((ijk >= 0) & (ijk < n), axis=2)
        ijk = np.clip(ijk, 0, n - 1)
    t = (ijk[..., 0] * n + ijk[..., 1]) * n + ijk[..., 2]
    occupied = np.zeros(n ** 3, bool)
    occupied[sites] = True
    return t, inside & ~occupied[t]


def propensities(kind, nu, beta, dU, valid):
    """r_j of every slot in FP64 (masked slots 0): kind 0 uniform 1, kind 1
    nu exp(-beta dU) (exponent capped at 600 so sums stay finite), kind 2
    nu min(1, exp(-beta dU))"""
    dU = np.asarray(dU, np.float64)
    valid = np.asarray(valid, bool)
    r = np.zeros(dU.shape)
    if kind == 0:
        r[valid] = 1.0
        return r
    x = -beta * dU[valid]
    if kind == 1:
        r[valid] = nu * np.exp(np.minimum(x, 600.0))
    elif kind == 2:
        r[valid] = np.where(x >= 0.0, nu, nu * np.exp(np.minimum(x, 0.0)))
    else:
        raise ValueError("rate kind must be 0, 1 or 2")
    return r


def cumulative(rates):
    """R_j = r_0 + ... + r_j, summed left to right (Alg. 1)"""
    return np.cumsum(np.asarray(rates, np.float64))


def select_slot(rates, T):
    """the j with R_{j-1} < T <= R_j (first such j); -1 if Q = 0 or T > Q"""
    R = cumulative(rates)
    if len(R) == 0 or R[-1] <= 0.0 or T > R[-1]:
        return -1
    return int(np.searchsorted(R, T, side="left"))


def time_increment(Q, xi):
    """Delta t = -log(xi) / Q (Alg. 1)"""
    return -np.log(xi) / Q if Q > 0 else np.inf
