/*
 * Lattice sums for the periodic far field (Sec. 2.2.1 "Periodic", Sec. 3.1
 * "Far-field component").  Test infrastructure only: see oracle.h.
 *
 * The operator R of the paper converts the multipole expansion of the primary
 * box into the local expansion (about the box centre) of the field of all its
 * periodic copies nu in V_inf = Z^3 \ {|nu_k| <= 1}.  It is the M2L operator
 * with Y_s^t(Q)/|Q|^{s+1} replaced by its sum over the copies Q = a nu.  With
 * box side a = 1 that sum is
 *     Lambda_s^t = sum_{nu in V_inf} Y_s^t(alpha_nu, beta_nu) / |nu|^{s+1}.
 *
 * This oracle computes it by brute force: the partial sums S(R) over complete
 * cubic shells 2 <= max_k |nu_k| <= R are taken for four radii, and the tail is
 * removed by Richardson extrapolation.  Because Y_s^t / r^{s+1} is harmonic,
 * replacing the sum over the unit cubes outside the cube of half-side R + 1/2
 * by the integral leaves only even-derivative corrections, so
 *     S(R) = Lambda - c1 (R+1/2)^{2-s} - c2 (R+1/2)^{-s-2} - c3 (R+1/2)^{-s-4} - ...
 * and four radii determine Lambda with an error of order (R+1/2)^{-s-6}.
 * For s = 0 the sum diverges (it multiplies the total charge, zero for a
 * neutral box) and for s = 1, 2 it is only conditionally convergent; odd s
 * vanish by inversion symmetry and s = 2 vanishes over every complete cubic
 * shell by cubic symmetry, so these entries are set to zero.  The dipole
 * term that cubic-shell summation leaves (App. B) is added by the caller.
 * Pinned in tests/test_oracle_lattice.py against an Ewald-split evaluation of
 * the same sums written independently in the test.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* sum over the complete cubic shell max_k |nu_k| = r of Y_s^t(nu)/|nu|^{s+1} */
static void shell_sum(int smax, int r, cplx *shell)
{
    int nt = (smax + 1) * (smax + 1);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * nt);
    memset(shell, 0, sizeof(cplx) * nt);
    for (int i = -r; i <= r; ++i)
        for (int j = -r; j <= r; ++j)
            for (int k = -r; k <= r; ++k) {
                int ai = abs(i), aj = abs(j), ak = abs(k);
                int mx = ai > aj ? ai : aj;
                if (ak > mx) mx = ak;
                if (mx != r) continue;
                double v[3] = {(double)i, (double)j, (double)k}, rho, th, ph;
                or_spherical(v, &rho, &th, &ph);
                or_sph_harmonics(smax, th, ph, Y);
                double inv = 1.0 / rho, rp = inv;
                for (int s = 0; s <= smax; ++s) {
                    for (int t = -s; t <= s; ++t) shell[or_idx(s, t)] += Y[or_idx(s, t)] * rp;
                    rp *= inv;
                }
            }
    free(Y);
}

/* solve the 4x4 system A x = b by Gaussian elimination with partial pivoting */
static void solve4(double A[4][4], double b[4], double x[4])
{
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int k = 0; k < 4; ++k) {
            double t = A[c][k];
            A[c][k] = A[piv][k];
            A[piv][k] = t;
        }
        double t = b[c];
        b[c] = b[piv];
        b[piv] = t;
        for (int r = c + 1; r < 4; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 4; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 3; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < 4; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
}

void or_lattice_sums(int smax, cplx *out)
{
    static const int radii[4] = {10, 14, 20, 28};
    int nt = (smax + 1) * (smax + 1);
    cplx *S[4];
    for (int q = 0; q < 4; ++q) {
        S[q] = (cplx *)calloc(nt, sizeof(cplx));
    }
    /* every shell once (independently, in parallel), then accumulated in
     * order of increasing radius with snapshots at the four radii */
    int rmax = radii[3];
    cplx *shells = (cplx *)calloc((size_t)(rmax + 1) * nt, sizeof(cplx));
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 2; r <= rmax; ++r) shell_sum(smax, r, shells + (size_t)r * nt);
    {
        cplx *acc = (cplx *)calloc(nt, sizeof(cplx));
        int q = 0;
        for (int r = 2; r <= rmax; ++r) {
            for (int i = 0; i < nt; ++i) acc[i] += shells[(size_t)r * nt + i];
            if (r == radii[q]) {
                memcpy(S[q], acc, sizeof(cplx) * nt);
                ++q;
            }
        }
        free(acc);
    }
    free(shells);
    for (int s = 0; s <= smax; ++s) {
        for (int t = -s; t <= s; ++t) {
            int id = or_idx(s, t);
            if (s < 3 || (s & 1)) {
                out[id] = 0.0;
                continue;
            }
            double A[4][4], bre[4], bim[4], xre[4], xim[4];
            for (int q = 0; q < 4; ++q) {
                double Rh = radii[q] + 0.5;
                double scale[4] = {1.0, pow(radii[0] + 0.5, s - 2.0), pow(radii[0] + 0.5, s + 2.0),
                                   pow(radii[0] + 0.5, s + 4.0)};
                A[q][0] = 1.0;
                A[q][1] = -pow(Rh, 2.0 - s) * scale[1];
                A[q][2] = -pow(Rh, -s - 2.0) * scale[2];
                A[q][3] = -pow(Rh, -s - 4.0) * scale[3];
                bre[q] = creal(S[q][id]);
                bim[q] = cimag(S[q][id]);
            }
            double A2[4][4];
            memcpy(A2, A, sizeof(A));
            solve4(A, bre, xre);
            solve4(A2, bim, xim);
            out[id] = xre[0] + I * xim[0];
        }
    }
    for (int q = 0; q < 4; ++q) free(S[q]);
}
