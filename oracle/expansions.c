/*
 * Multipole and local expansions and the three translation operators T_MM,
 * T_ML, T_LL of Sec. 2.2 (definitions list) and Alg. "fmm" (App. A), written in
 * the classical complex form of Greengard and Rokhlin (the paper takes the
 * operators from that literature and does not print them).  Test
 * infrastructure only: see oracle.h.
 *
 * With A_n^m = (-1)^n / sqrt((n-m)!(n+m)!):
 *   P2M  M_n^m = sum_i q_i rho_i^n Y_n^{-m}(alpha_i, beta_i)
 *   M2M  M_j^k = sum_{n<=j} sum_m O_{j-n}^{k-m} i^{|k|-|m|-|k-m|} A_n^m A_{j-n}^{k-m}
 *                 rho^n Y_n^{-m}(alpha,beta) / A_j^k
 *   M2L  L_j^k = sum_{n<=p} sum_m O_n^m i^{|k-m|-|k|-|m|} A_n^m A_j^k
 *                 Y_{j+n}^{m-k}(alpha,beta) / ((-1)^n A_{j+n}^{m-k} rho^{j+n+1})
 *   L2L  L_j^k = sum_{n>=j} sum_m O_n^m i^{|m|-|m-k|-|k|} A_{n-j}^{m-k} A_j^k
 *                 Y_{n-j}^{m-k}(alpha,beta) rho^{n-j} / ((-1)^{n+j} A_n^m)
 *   P2L  L_n^m = q Y_n^{-m}(alpha,beta) / rho^{n+1}
 * where (rho, alpha, beta) are the spherical coordinates of the displacement Q
 * named at each function.  The index-only factors (i-powers and A's) of each
 * operator are tabulated once per order p in an or_ops; nothing else is
 * precomputed or reordered.  Pinned in tests/test_oracle_expansions.py against
 * direct Coulomb sums (P2M, M2L, P2L within the truncation bound; M2M and L2L
 * exact for truncated expansions).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

double or_A(int n, int m)
{
    int am = abs(m);
    double prod = 1.0;                       /* (n-m)!(n+m)! */
    for (int k = 2; k <= n - am; ++k) prod *= (double)k;
    for (int k = 2; k <= n + am; ++k) prod *= (double)k;
    return ((n & 1) ? -1.0 : 1.0) / sqrt(prod);
}

cplx or_ipow(int e)
{
    int r = ((e % 4) + 4) % 4;
    switch (r) {
    case 0: return 1.0;
    case 1: return I;
    case 2: return -1.0;
    default: return -I;
    }
}

or_ops *or_ops_create(int p)
{
    or_ops *o = (or_ops *)calloc(1, sizeof(or_ops));
    int nt = (p + 1) * (p + 1);
    o->p = p;
    o->nt = nt;
    o->fmm = (cplx *)calloc((size_t)nt * nt, sizeof(cplx));
    o->fml = (cplx *)calloc((size_t)nt * nt, sizeof(cplx));
    o->fll = (cplx *)calloc((size_t)nt * nt, sizeof(cplx));
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k)
            for (int n = 0; n <= p; ++n)
                for (int m = -n; m <= n; ++m) {
                    size_t at = (size_t)or_idx(j, k) * nt + or_idx(n, m);
                    if (n <= j && abs(k - m) <= j - n)
                        o->fmm[at] = or_ipow(abs(k) - abs(m) - abs(k - m)) * or_A(n, m) *
                                     or_A(j - n, k - m) / or_A(j, k);
                    o->fml[at] = or_ipow(abs(k - m) - abs(k) - abs(m)) * or_A(n, m) * or_A(j, k) /
                                 (((n & 1) ? -1.0 : 1.0) * or_A(j + n, m - k));
                    if (n >= j && abs(m - k) <= n - j)
                        o->fll[at] = or_ipow(abs(m) - abs(m - k) - abs(k)) * or_A(n - j, m - k) *
                                     or_A(j, k) / ((((n + j) & 1) ? -1.0 : 1.0) * or_A(n, m));
                }
    return o;
}

void or_ops_destroy(or_ops *o)
{
    if (!o) return;
    free(o->fmm);
    free(o->fml);
    free(o->fll);
    free(o);
}

/* rho^n Y_n^m(alpha, beta) and Y_n^m(alpha, beta) / rho^{n+1} of a displacement */
static void regular_of(int nmax, const double d[3], cplx *out)
{
    double rho, al, be;
    or_spherical(d, &rho, &al, &be);
    or_sph_harmonics(nmax, al, be, out);
    double rn = 1.0;
    for (int n = 0; n <= nmax; ++n) {
        for (int m = -n; m <= n; ++m) out[or_idx(n, m)] *= rn;
        rn *= rho;
    }
}

static void irregular_of(int nmax, const double d[3], cplx *out)
{
    double rho, al, be;
    or_spherical(d, &rho, &al, &be);
    or_sph_harmonics(nmax, al, be, out);
    double inv = 1.0 / rho, rp = inv;
    for (int n = 0; n <= nmax; ++n) {
        for (int m = -n; m <= n; ++m) out[or_idx(n, m)] *= rp;
        rp *= inv;
    }
}

void ops_p2m_add(const or_ops *o, double q, const double d[3], cplx *M, cplx *scratch)
{
    /* d = position - centre */
    regular_of(o->p, d, scratch);
    for (int n = 0; n <= o->p; ++n)
        for (int m = -n; m <= n; ++m) M[or_idx(n, m)] += q * scratch[or_idx(n, -m)];
}

void ops_m2m(const or_ops *o, const cplx *O, const double Q[3], cplx *M, cplx *scratch)
{
    int p = o->p, nt = o->nt;
    regular_of(p, Q, scratch);
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
            cplx s = 0.0;
            const cplx *f = o->fmm + (size_t)or_idx(j, k) * nt;
            for (int n = 0; n <= j; ++n)
                for (int m = -n; m <= n; ++m) {
                    if (abs(k - m) > j - n) continue;
                    s += O[or_idx(j - n, k - m)] * f[or_idx(n, m)] * scratch[or_idx(n, -m)];
                }
            M[or_idx(j, k)] = s;
        }
}

void ops_m2l_add(const or_ops *o, const cplx *O, const double Q[3], cplx *L, cplx *scratch2p)
{
    int p = o->p, nt = o->nt;
    irregular_of(2 * p, Q, scratch2p);
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
            cplx s = 0.0;
            const cplx *f = o->fml + (size_t)or_idx(j, k) * nt;
            for (int n = 0; n <= p; ++n)
                for (int m = -n; m <= n; ++m)
                    s += O[or_idx(n, m)] * f[or_idx(n, m)] * scratch2p[or_idx(j + n, m - k)];
            L[or_idx(j, k)] += s;
        }
}

/* The same contraction with the geometric factor G_s^t = Y_s^t / rho^{s+1}
 * supplied by the caller (used for the lattice-sum operator R). */
void ops_m2l_with_geometry(const or_ops *o, const cplx *O, const cplx *G, cplx *L)
{
    int p = o->p, nt = o->nt;
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
            cplx s = 0.0;
            const cplx *f = o->fml + (size_t)or_idx(j, k) * nt;
            for (int n = 0; n <= p; ++n)
                for (int m = -n; m <= n; ++m)
                    s += O[or_idx(n, m)] * f[or_idx(n, m)] * G[or_idx(j + n, m - k)];
            L[or_idx(j, k)] += s;
        }
}

void ops_l2l_add(const or_ops *o, const cplx *O, const double Q[3], cplx *L, cplx *scratch)
{
    int p = o->p, nt = o->nt;
    regular_of(p, Q, scratch);
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
            cplx s = 0.0;
            const cplx *f = o->fll + (size_t)or_idx(j, k) * nt;
            for (int n = j; n <= p; ++n)
                for (int m = -n; m <= n; ++m) {
                    if (abs(m - k) > n - j) continue;
                    s += O[or_idx(n, m)] * f[or_idx(n, m)] * scratch[or_idx(n - j, m - k)];
                }
            L[or_idx(j, k)] += s;
        }
}

void ops_p2l_add(const or_ops *o, double q, const double d[3], cplx *L, cplx *scratch)
{
    /* d = source - centre */
    irregular_of(o->p, d, scratch);
    for (int n = 0; n <= o->p; ++n)
        for (int m = -n; m <= n; ++m) L[or_idx(n, m)] += q * scratch[or_idx(n, -m)];
}

double ops_eval_local(const or_ops *o, const cplx *L, const double d[3], cplx *scratch)
{
    /* d = point - centre */
    regular_of(o->p, d, scratch);
    cplx s = 0.0;
    for (int i = 0; i < o->nt; ++i) s += L[i] * scratch[i];
    return creal(s);
}

/* ---- public single-shot wrappers (used by the pin tests) ---------------- */

void or_p2m(int p, int n, const double *xyz, const double *q, const double c[3], cplx *M)
{
    or_ops *o = or_ops_create(p);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * o->nt);
    memset(M, 0, sizeof(cplx) * o->nt);
    for (int i = 0; i < n; ++i) {
        double d[3] = {xyz[3 * i] - c[0], xyz[3 * i + 1] - c[1], xyz[3 * i + 2] - c[2]};
        ops_p2m_add(o, q[i], d, M, Y);
    }
    free(Y);
    or_ops_destroy(o);
}

void or_m2m(int p, const cplx *O, const double Q[3], cplx *M)
{
    or_ops *o = or_ops_create(p);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * o->nt);
    ops_m2m(o, O, Q, M, Y);
    free(Y);
    or_ops_destroy(o);
}

void or_m2l(int p, const cplx *O, const double Q[3], cplx *L)
{
    or_ops *o = or_ops_create(p);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * (2 * p + 1) * (2 * p + 1));
    memset(L, 0, sizeof(cplx) * o->nt);
    ops_m2l_add(o, O, Q, L, Y);
    free(Y);
    or_ops_destroy(o);
}

void or_l2l(int p, const cplx *O, const double Q[3], cplx *L)
{
    or_ops *o = or_ops_create(p);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * o->nt);
    memset(L, 0, sizeof(cplx) * o->nt);
    ops_l2l_add(o, O, Q, L, Y);
    free(Y);
    or_ops_destroy(o);
}

void or_p2l(int p, double q, const double src[3], const double c[3], cplx *L)
{
    or_ops *o = or_ops_create(p);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * o->nt);
    double d[3] = {src[0] - c[0], src[1] - c[1], src[2] - c[2]};
    memset(L, 0, sizeof(cplx) * o->nt);
    ops_p2l_add(o, q, d, L, Y);
    free(Y);
    or_ops_destroy(o);
}

double or_eval_multipole(int p, const cplx *M, const double c[3], const double x[3])
{
    int nt = (p + 1) * (p + 1);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * nt);
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    irregular_of(p, d, Y);
    cplx s = 0.0;
    for (int i = 0; i < nt; ++i) s += M[i] * Y[i];
    free(Y);
    return creal(s);
}

double or_eval_local(int p, const cplx *L, const double c[3], const double x[3])
{
    or_ops *o = or_ops_create(p);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * o->nt);
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double v = ops_eval_local(o, L, d, Y);
    free(Y);
    or_ops_destroy(o);
    return v;
}
