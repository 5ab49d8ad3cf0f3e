/*
 * CPU oracle for FMM-based electrostatics in kinetic Monte Carlo
 * (Saunders, Grant, Mueller, Thompson, "Fast electrostatic solvers for kinetic
 * Monte Carlo simulations", arXiv:1905.04065).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is a plain, slow, FP64 statement of what
 * the method computes.  It exists so the GPU library can be checked against it.
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant generator with the
 * GPU library, and the GPU library never calls it.
 *
 * Two oracles live here:
 *   O-exact  plain definitions: the direct pair sum of the Coulomb energy (the
 *            pair-loop energy of Sec. 5.1) and, for periodic boxes, Ewald
 *            summation with conducting ("tin-foil") surroundings.
 *   O-fmm    the FMM-KMC method of Sec. 3 taken step by step in the paper's
 *            notation: Alg. "fmm" (App. A) for the fine-level local expansions,
 *            Eq. (proposed_energy) / Eq. (proposed_energy_sr) plus the far-field
 *            E, K, H bookkeeping of Sec. 3.1 for a proposal, and the accept step
 *            of Sec. 3 / Sec. 3.1.
 *
 * Harmonics follow the classical FMM normalisation
 *     Y_n^m(theta,phi) = sqrt((n-|m|)!/(n+|m|)!) P_n^{|m|}(cos theta) e^{i m phi}
 * with P_n^m the associated Legendre functions without the Condon-Shortley
 * phase, so that the expansions read exactly as Eq. (multipole_local_expansion):
 *     Phi = sum M_n^m r^{-(n+1)} Y_n^m,     Psi = sum L_n^m r^n Y_n^m.
 * Coefficient (n,m), -n <= m <= n, is stored at index n*n + n + m.
 *
 * Every function with a numerical result is pinned by a CPU test against
 * something other than itself (direct sums, closed forms, invariants, brute
 * force); see the test files named in each section below.
 */
#ifndef FMMKMC_ORACLE_H
#define FMMKMC_ORACLE_H

#include <stdint.h>
#include <complex.h>

typedef double _Complex cplx;

static inline int or_idx(int n, int m) { return n * n + n + m; }

/* ---- harmonics (harmonics.c) ------------------------------------------ */
/* Y_n^m(theta, phi) for 0 <= n <= nmax, all m; out has (nmax+1)^2 entries. */
void or_sph_harmonics(int nmax, double theta, double phi, cplx *out);
/* Spherical coordinates (r, theta, phi) of v; theta = phi = 0 at the origin. */
void or_spherical(const double v[3], double *r, double *theta, double *phi);

/* ---- expansions (expansions.c) --------------------------------------- */
/* A_n^m = (-1)^n / sqrt((n-m)!(n+m)!) */
double or_A(int n, int m);
/* i^e for an integer e */
cplx or_ipow(int e);
void or_p2m(int p, int n, const double *xyz, const double *q, const double c[3], cplx *M);
void or_m2m(int p, const cplx *O, const double Q[3], cplx *M);          /* Q = old - new centre */
void or_m2l(int p, const cplx *O, const double Q[3], cplx *L);          /* Q = source - target centre */
void or_l2l(int p, const cplx *O, const double Q[3], cplx *L);          /* Q = old - new centre */
void or_p2l(int p, double q, const double src[3], const double c[3], cplx *L);
double or_eval_multipole(int p, const cplx *M, const double c[3], const double x[3]);
double or_eval_local(int p, const cplx *L, const double c[3], const double x[3]);

/* ---- lattice sums (lattice.c) ----------------------------------------- */
/* Lambda_s^t = sum_{nu in V_inf} Y_s^t(angles of nu) / |nu|^{s+1}  (box a = 1),
 * V_inf = Z^3 minus {|nu_k| <= 1}.  Entries s < 3 and odd s are zero by the
 * cubic symmetry of complete cubic shells.  out has (smax+1)^2 entries. */
void or_lattice_sums(int smax, cplx *out);

/* ---- exact sums (exact.c) -------------------------------------------- */
double or_direct_energy(int n, const double *xyz, const double *q);
void or_direct_dU(int n, const double *xyz, const double *q, int np,
                  const int64_t *idx, const double *tgt, double *dU);
double or_ewald_energy(int n, const double *xyz, const double *q, double a,
                       double alpha, double rc, double kc);
void or_ewald_dU(int n, const double *xyz, const double *q, double a, double alpha,
                 double rc, double kc, int np, const int64_t *idx, const double *tgt,
                 double *dU);
/* psi_self - psi(d) of a unit charge and its own copies (tin-foil Ewald) */
double or_periodic_self_change(double a, const double d[3]);

/* ---- O-fmm (fmm_kmc.c) ------------------------------------------------ */
typedef struct of_ctx of_ctx;
/* bc: 0 free space, 1 periodic.  L: number of levels, root = level 1.
 * lazy: 0 computes Psi_L for every fine cell at initialise, 1 computes the
 * fine-level local expansion of a cell on first use (same operations, same
 * order, restricted to the cells that are asked for). */
of_ctx *of_create(int bc, double a, int L, int p, int n, const double *xyz,
                  const double *q, int lazy);
/* as of_create; per_level: keep the local expansion of every level apart (the
 * interaction-list terms of that level only) and apply the accept rule per
 * level (see fmm_kmc.c) */
of_ctx *of_create_levels(int bc, double a, int L, int p, int n, const double *xyz, const double *q, int lazy,
                         int per_level);
void of_destroy(of_ctx *c);
/* self-image terms of a periodic proposal: 0 (default) the paper's V_box sum,
 * constant and 1/2 dE.R'dK (Sec. 3.1); 1 the exact change q^2 (psi_self -
 * psi(r' - r)) of the moving charge's interaction with its own copies */
void of_set_self_image(of_ctx *c, int exact);
/* uniform external field E: every proposal adds -q E.d, d the hop (periodic:
 * minimum image) */
void of_set_field(of_ctx *c, const double E[3]);
double of_energy(of_ctx *c);
void of_propose(of_ctx *c, int np, const int64_t *idx, const double *tgt, double *dU);
double of_accept(of_ctx *c, int64_t i, const double newpos[3]);
int of_nterms(of_ctx *c);
int of_fine_cell_of(of_ctx *c, const double x[3]);
void of_get_local(of_ctx *c, int cell, cplx *out);
void of_get_multipole(of_ctx *c, int level, int cell, cplx *out);
void of_get_level_local(of_ctx *c, int level, int cell, cplx *out);
void of_get_far(of_ctx *c, cplx *E, cplx *K, cplx *H);
void of_get_positions(of_ctx *c, double *xyz);
double of_potential(of_ctx *c, const double x[3], int64_t exclude);
void of_rebuild_multipoles(of_ctx *c, int level, int cell, cplx *out);

#endif
