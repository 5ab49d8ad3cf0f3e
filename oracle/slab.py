"""Charges between two grounded plates (Sec. 2.2.2, "Dirichlet").

TEST INFRASTRUCTURE ONLY (like the rest of this package): the plain statement
of what the slab mode of the GPU library computes, used to check it.

The paper imposes zero potential on the top and bottom of the domain by
extending the physical charges with their first mirror image and treating the
extended domain with the periodic algorithm.  Here the physical slab is
[0, a) x [0, a) x [0, a/2); each charge q at (x, y, z) gets the mirror -q at
(x, y, a - z); the doubled system is periodic with period a in all three
directions (conducting boundary, as the periodic oracle).  The doubled charge
distribution is odd under z -> -z and z -> a - z, so its periodic potential
vanishes on the planes z = 0 and z = a/2.

Energies and moves of the physical system:
  * U_phys = U_doubled / 2 - E_z sum q z (every physical interaction appears
    twice in the doubled system; a uniform field E_z along z adds -E_z q z);
  * a hop of charge i moves its mirror m as well:
      dU_pair = dU_i + dU_m + q_i q_m [G(ri'-rm') - G(ri'-rm) - G(ri-rm') + G(ri-rm)],
    dU_i and dU_m being single moves with the partner at its old place and G
    the periodic pair potential (the bracket corrects the partner term);
    dU_phys = dU_pair / 2 - E_z q_i dz.
The single moves come from O-fmm (or O-exact); the bracket from the Ewald pair
potential of O-exact.
"""
import numpy as np

from . import FmmKmc, ewald_dU


def mirror_system(xyz, q, a):
    """the doubled system: physical charges 0..N-1, mirrors N..2N-1"""
    xyz = np.asarray(xyz, np.float64).reshape(-1, 3)
    q = np.asarray(q, np.float64).reshape(-1)
    mir = xyz.copy()
    mir[:, 2] = a - xyz[:, 2]
    return np.vstack([xyz, mir]), np.concatenate([q, -q])


def mirror_point(x, a):
    x = np.asarray(x, np.float64).reshape(3).copy()
    x[2] = a - x[2]
    return x


def pair_bracket(ri, rm, ri_new, rm_new, a):
    """G(ri'-rm') - G(ri'-rm) - G(ri-rm') + G(ri-rm) with the Ewald pair potential:
    each difference G(ri'-r) - G(ri-r) is the Ewald dU of moving a unit charge
    from ri to ri' beside a unit charge at r"""
    A = ewald_dU(np.vstack([ri, rm_new]), [1.0, 1.0], a, [0], [ri_new])[0]
    B = ewald_dU(np.vstack([ri, rm]), [1.0, 1.0], a, [0], [ri_new])[0]
    return A - B


class SlabOracle:
    """The slab on top of O-fmm (the doubled periodic system, same L and p as
    the GPU run); hops given as target positions of physical charges."""

    def __init__(self, xyz, q, a, L, p, ez=0.0):
        self.a, self.ez = float(a), float(ez)
        self.N = len(np.asarray(q).reshape(-1))
        xyz2, q2 = mirror_system(xyz, q, self.a)
        self.fmm = FmmKmc(xyz2, q2, self.a, L, p, "periodic")
        self.q = q2[: self.N].copy()

    def positions(self):
        return self.fmm.positions()[: self.N]

    @property
    def energy(self):
        z = self.positions()[:, 2]
        return 0.5 * self.fmm.energy - self.ez * float(np.dot(self.q, z))

    def propose(self, i, target):
        pos = self.fmm.positions()
        ri, rm = pos[i], pos[self.N + i]
        t = np.asarray(target, np.float64).reshape(3)
        tm = mirror_point(t, self.a)
        du_i = self.fmm.propose([i], [t])[0]
        du_m = self.fmm.propose([self.N + i], [tm])[0]
        qi = self.q[i]
        X = qi * (-qi) * pair_bracket(ri, rm, t, tm, self.a)
        return 0.5 * (du_i + du_m + X) - self.ez * qi * (t[2] - ri[2])

    def accept(self, i, target):
        z_old = self.fmm.positions()[i, 2]
        t = np.asarray(target, np.float64).reshape(3)
        d1 = self.fmm.accept(i, t)
        d2 = self.fmm.accept(self.N + i, mirror_point(t, self.a))
        return 0.5 * (d1 + d2) - self.ez * self.q[i] * (t[2] - z_old)
