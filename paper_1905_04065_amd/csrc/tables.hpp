// Host-side construction of geometry-only constant tables: translation
// operators as real (p+1)^2 x (p+1)^2 matrices, the periodic far-field operator
// R (lattice sums plus dipole term), the Chebyshev map of the far-field
// potential and the lattice tables of the 2x2x2-sites-per-cell fast path.
// Nothing here depends on the charges; all charge-dependent arithmetic runs in
// the HIP kernels.
#pragma once

#include <complex>
#include <vector>

namespace fmmkmc {

using cplx = std::complex<double>;

// full complex harmonics, index n*n + n + m, n <= nmax
void regular_all(int nmax, double x, double y, double z, cplx *out);
void irregular_all(int nmax, double x, double y, double z, cplx *out);

// Matrices act on real-stored expansions: out[k] = sum_n mat[k * nt + n] in[n].
// M2M: child multipole about the child centre -> parent centre; s = child - parent.
void build_m2m(int p, double sx, double sy, double sz, double *mat);
// L2L: parent local -> child centre; s = child - parent.
void build_l2l(int p, double sx, double sy, double sz, double *mat);
// M2L: source multipole -> target local; d = target centre - source centre.
void build_m2l(int p, double dx, double dy, double dz, double *mat);

// S_s^t = sum over copies nu in V_inf = Z^3 \ {|nu_k| <= 1} of I_s^t(a nu),
// s <= smax, by Ewald splitting of the lattice sum of a homogeneous harmonic
// polynomial; entries with s < 3 or odd s are zero (cubic symmetry).
void lattice_sums(int smax, double a, cplx *S);
// H = R K for the copies in V_inf, including the dipole term -(4 pi / 3V) M.(x - c)
// of the conducting-boundary convention (App. B of the paper).
void build_far_operator(int p, double a, double *mat);

// Chebyshev map: the far-field potential Psi(x) = sum_k H_k w_k(x - c),
// c = (a/2)(1,1,1), equals sum_{abc} C_abc T_a(xi) T_b(eta) T_c(zeta) with
// (xi, eta, zeta) = (x - c) / (a/2) and C = G H, G of shape (p+1)^3 x nt.
// Returns the largest coefficient that should vanish (total degree > p).
double build_cheb_map(int p, double a, double *G);

// 2x2x2-sites-per-cell lattice: L2P weights at the 8 sites of a cell
// (u = 4 lx + 2 ly + lz), and the 1/r table from the 8 sites to the 216 sites
// of the 27-cell block (v = 8 nb + u', nb = 9(dx+1) + 3(dy+1) + (dz+1)).
void build_s2_tables(int p, double h, double *Y2, double *T2);

}  // namespace fmmkmc
