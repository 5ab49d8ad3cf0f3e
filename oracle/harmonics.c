/*
 * Spherical harmonics in the classical FMM normalisation (the Y_n^m of
 * Eq. (multipole_local_expansion)).  Test infrastructure only: see oracle.h.
 *
 * Associated Legendre functions without the Condon-Shortley phase, by the
 * textbook three-term recurrence in n at fixed m:
 *     P_m^m(x)     = (2m-1)!! (1-x^2)^{m/2}
 *     P_{m+1}^m(x) = (2m+1) x P_m^m(x)
 *     (n-m) P_n^m  = (2n-1) x P_{n-1}^m - (n+m-1) P_{n-2}^m
 * Pinned in tests/test_oracle_expansions.py against closed forms of the
 * low-degree harmonics and against the Legendre addition theorem.
 */
#include <math.h>
#include <stdlib.h>
#include "oracle.h"

void or_spherical(const double v[3], double *r, double *theta, double *phi)
{
    double rr = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    *r = rr;
    if (rr == 0.0) {
        *theta = 0.0;
        *phi = 0.0;
        return;
    }
    double c = v[2] / rr;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    *theta = acos(c);
    *phi = atan2(v[1], v[0]);
}

/* sqrt((n-m)!/(n+m)!) as 1/sqrt of the product (n-m+1)...(n+m) */
static double ynorm(int n, int am)
{
    double prod = 1.0;
    for (int k = n - am + 1; k <= n + am; ++k) prod *= (double)k;
    return 1.0 / sqrt(prod);
}

void or_sph_harmonics(int nmax, double theta, double phi, cplx *out)
{
    int w = nmax + 1;
    double *P = (double *)calloc((size_t)w * w, sizeof(double));
    double x = cos(theta), s = sin(theta);
    if (s < 0) s = -s;
    P[0] = 1.0;
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) P[m * w + m] = (2.0 * m - 1.0) * s * P[(m - 1) * w + (m - 1)];
        if (m + 1 <= nmax) P[(m + 1) * w + m] = (2.0 * m + 1.0) * x * P[m * w + m];
        for (int n = m + 2; n <= nmax; ++n)
            P[n * w + m] = ((2.0 * n - 1.0) * x * P[(n - 1) * w + m] -
                            (n + m - 1.0) * P[(n - 2) * w + m]) / (double)(n - m);
    }
    for (int n = 0; n <= nmax; ++n) {
        for (int m = -n; m <= n; ++m) {
            int am = abs(m);
            double norm = ynorm(n, am);
            out[or_idx(n, m)] = norm * P[n * w + am] * cexp(I * (double)m * phi);
        }
    }
    free(P);
}
