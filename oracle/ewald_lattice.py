"""O-exact for charges on a periodic site lattice: tin-foil Ewald energy changes
at lattice sizes the pair-by-pair Ewald sum of exact.c cannot reach.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The conducting-boundary periodic pair potential (the exactly periodic
potential of the dipole condition of Sec. 2.2.2 / App. B, Ewald summation as
the paper's reference method in Sec. 1 and Sec. 4)
    psi(x) = sum_nu erfc(alpha |x + a nu|) / |x + a nu|
           + (4 pi / V) sum_{k != 0} exp(-k^2 / 4 alpha^2) / k^2 cos(k . x)   (+ const)
gives for a move of charge i from site r to site t
    dU = q_i sum_{j != i} q_j (psi(t - r_j) - psi(r - r_j)).
Reciprocal part: with Phi(x) = sum_j q_j psi_k(x - r_j) (all charges) it is
q_i [Phi(t) - Phi(r) - q_i (psi_k(t - r) - psi_k(0))].  On the lattice, Phi at
every site is a cyclic convolution of the site charges with psi_k, taken with
a 3-D FFT (numpy); alpha is small enough (alpha h = 1/4) that every wave
vector beyond the lattice's own (|k| >= pi / h) weighs below 1e-17, so the
lattice's finite set of wave vectors loses nothing.  Real part: the sum over
the charges within r_c = 5.9 / alpha of t and of r (erfc(5.9) < 1e-16).

Pinned in tests/test_oracle_exact.py against the pair-by-pair Ewald sum of
exact.c on small lattices and by independence of alpha.
"""
import numpy as np
from scipy.special import erfc


class LatticeEwald:
    """sites: lattice index (i n + j) n + k of each charge; n sites per axis,
    spacing h (box a = n h); q: charges (sum 0)."""

    def __init__(self, sites, q, n, h=1.0, alpha_h=0.25, cut=5.9):
        self.n, self.h = int(n), float(h)
        self.a = self.n * self.h
        self.alpha = alpha_h / self.h
        self.rc = cut / self.alpha
        sites = np.asarray(sites, np.int64)
        self.q = np.asarray(q, np.float64)
        self.sites = sites.copy()
        n_ = self.n
        grid = np.zeros(n_ ** 3)
        grid[sites] = self.q
        self.grid = grid.reshape(n_, n_, n_)
        # reciprocal kernel: exp(-k^2 / 4 alpha^2) / k^2 on the centred frequencies, 0 at k = 0
        m = np.fft.fftfreq(n_) * n_
        kx, ky, kz = np.meshgrid(m, m, m, indexing="ij")
        k2 = (2.0 * np.pi / self.a) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            G = np.where(k2 > 0, np.exp(-k2 / (4.0 * self.alpha ** 2)) / k2, 0.0)
        V = self.a ** 3
        self.G = G
        pref = 4.0 * np.pi / V * n_ ** 3
        self.phi_k = np.real(np.fft.ifftn(np.fft.fftn(self.grid) * G)) * pref  # Phi at every site
        # psi_k(d) for a lattice displacement d: the same convolution with a unit charge at the origin
        self.psi_k_grid = np.real(np.fft.ifftn(G)) * pref
        # real-space stencil: lattice offsets within rc (nearest image is enough: rc < a / 2 is not
        # required, images are handled by wrapping the offsets)
        R = int(np.ceil(self.rc / self.h))
        o = np.arange(-R, R + 1)
        ox, oy, oz = np.meshgrid(o, o, o, indexing="ij")
        d = self.h * np.sqrt(ox ** 2 + oy ** 2 + oz ** 2)
        keep = (d <= self.rc) & (d > 0)
        self.off = np.stack([ox[keep], oy[keep], oz[keep]], 1)
        self.w_off = erfc(self.alpha * d[keep]) / d[keep]
        self.occ = np.zeros(n_ ** 3, np.int64) - 1
        self.occ[sites] = np.arange(len(sites))

    def _ijk(self, s):
        n = self.n
        return np.array([s // (n * n), (s // n) % n, s % n])

    def _real_phi(self, s, exclude):
        """real-space potential at site s from every charge except `exclude`
        (their copies too; the stencil must stay within one period)"""
        n = self.n
        ijk = self._ijk(s)[None, :] + self.off
        ijk %= n
        idx = (ijk[:, 0] * n + ijk[:, 1]) * n + ijk[:, 2]
        j = self.occ[idx]
        qj = np.where(j >= 0, self.q[np.maximum(j, 0)], 0.0)
        qj = np.where(j == exclude, 0.0, qj)
        return float(np.dot(qj, self.w_off))

    def dU(self, i, t_site):
        """energy change of moving charge i to the (vacant) site t_site"""
        i = int(i)
        r_site = int(self.sites[i])
        t_site = int(t_site)
        qi = self.q[i]
        n = self.n
        # real space: the other charges (every image within rc) at t and at r
        real = self._real_phi(t_site, i) - self._real_phi(r_site, i)
        # reciprocal space: Phi holds charge i at r; take its term out at both points
        dk = (self._ijk(t_site) - self._ijk(r_site)) % n
        phi = self.phi_k.reshape(-1)
        recip = (phi[t_site] - qi * self.psi_k_grid[dk[0], dk[1], dk[2]]) - (phi[r_site] - qi * self.psi_k_grid[0, 0, 0])
        return qi * (real + recip)

    def dU_many(self, idx, t_sites):
        return np.array([self.dU(i, t) for i, t in zip(idx, t_sites)])
