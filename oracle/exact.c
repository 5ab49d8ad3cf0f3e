/*
 * O-exact: plain definitions of the electrostatic energy and of its change for
 * a single-charge move.  Test infrastructure only: see oracle.h.
 *
 * Free space: the pair sum U = 1/2 sum_{i != j} q_i q_j / |r_i - r_j| of
 * Eq. (naive_coulomb) (Sec. 5.1), and for a move of charge i from r to r'
 *     dU = q_i sum_{j != i} q_j (1/|r' - r_j| - 1/|r - r_j|).
 *
 * Periodic: Ewald summation (cited in Sec. 1 and Sec. 4 as the reference method)
 * with conducting surroundings, i.e. the exactly periodic potential the paper
 * asks for with its dipole condition (Sec. 2.2.2, App. B):
 *     psi(x) = sum_nu erfc(alpha|x + a nu|)/|x + a nu|
 *            + (4 pi / V) sum_{k != 0} exp(-k^2/(4 alpha^2)) / k^2 cos(k.x) - pi/(alpha^2 V)
 *     U  = 1/2 sum_{i != j} q_i q_j psi(r_i - r_j) + 1/2 sum_i q_i^2 psi_self
 *     psi_self = lim_{x->0} (psi(x) - 1/|x|)
 *     dU = q_i sum_{j != i} q_j (psi(r' - r_j) - psi(r - r_j))
 * (a charge's interaction with its own copies does not depend on where it is).
 *
 * or_periodic_self_change(a, d) = psi_self - psi(d): the change of a unit
 * charge's interaction with its own periodic copies when it is displaced by d
 * while the copies stay where they were.  A KMC proposal's FMM potential
 * difference q (phi(r') - phi(r)) contains this term for the moving charge
 * (its copies sit at the old place); adding q^2 (psi_self - psi(d)) removes it
 * exactly, which is the exact counterpart of the V_box self terms plus the
 * quadratic far-field term of Sec. 3.1.  Pinned by the caesium chloride
 * Madelung constant (d = half the body diagonal) and by the small-d expansion
 * psi(d) = 1/|d| + psi_self + (2 pi / 3V) |d|^2 + O(|d|^4 / a^5).
 * alpha, the real-space cutoff rc and the reciprocal cutoff kc are chosen by the
 * caller; the result is independent of alpha to rounding when both truncation
 * errors are below it.  Pinned in tests/test_oracle_exact.py by the Madelung
 * constants of rock salt and caesium chloride, by independence of alpha, and
 * by the direct pair sum over a large cube of copies for a neutral pair.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

double or_direct_energy(int n, const double *xyz, const double *q)
{
    double U = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (i == j) continue;
            double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
                   dz = xyz[3 * i + 2] - xyz[3 * j + 2];
            U += 0.5 * q[i] * q[j] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return U;
}

void or_direct_dU(int n, const double *xyz, const double *q, int np, const int64_t *idx,
                  const double *tgt, double *dU)
{
#pragma omp parallel for schedule(static)
    for (int s = 0; s < np; ++s) {
        int64_t i = idx[s];
        const double *t = tgt + 3 * s, *r = xyz + 3 * i;
        double acc = 0.0;
        int bad = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const double *rj = xyz + 3 * j;
            double a0 = t[0] - rj[0], a1 = t[1] - rj[1], a2 = t[2] - rj[2];
            double b0 = r[0] - rj[0], b1 = r[1] - rj[1], b2 = r[2] - rj[2];
            double dn = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
            if (dn == 0.0) bad = 1;
            acc += q[j] * (1.0 / dn - 1.0 / sqrt(b0 * b0 + b1 * b1 + b2 * b2));
        }
        dU[s] = bad ? NAN : q[i] * acc;
    }
}

/* ---- Ewald ---------------------------------------------------------------- */

typedef struct {
    double a, alpha, rc, kc, V;
    int nimg;      /* real-space copies |nu_k| <= nimg */
    int nk;        /* reciprocal vectors 2 pi m / a with |m_k| <= nk */
} ewald_par;

static ewald_par ewald_setup(double a, double alpha, double rc, double kc)
{
    ewald_par e;
    e.a = a;
    e.alpha = alpha;
    e.rc = rc;
    e.kc = kc;
    e.V = a * a * a;
    e.nimg = (int)ceil(rc / a) + 1;
    e.nk = (int)ceil(kc * a / (2.0 * M_PI));
    return e;
}

/* compensated (Kahan) accumulation: the sums below add up to ~10^6 terms whose
 * total largely cancels against the self term */
static void kadd(double *s, double *c, double v)
{
    double y = v - *c, t = *s + y;
    *c = (t - *s) - y;
    *s = t;
}

/* real-space part of psi(x), excluding the singular term at the origin when
 * skip_origin is set */
static double ewald_real(const ewald_par *e, const double x[3], int skip_origin)
{
    double s = 0.0, comp = 0.0;
    for (int i = -e->nimg; i <= e->nimg; ++i)
        for (int j = -e->nimg; j <= e->nimg; ++j)
            for (int k = -e->nimg; k <= e->nimg; ++k) {
                if (skip_origin && i == 0 && j == 0 && k == 0) continue;
                double d0 = x[0] + e->a * i, d1 = x[1] + e->a * j, d2 = x[2] + e->a * k;
                double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                if (r > e->rc) continue;
                kadd(&s, &comp, erfc(e->alpha * r) / r);
            }
    return s;
}

/* reciprocal-space part of psi(x) (without the constant) */
static double ewald_recip(const ewald_par *e, const double x[3])
{
    double s = 0.0, comp = 0.0, g = 2.0 * M_PI / e->a;
    for (int i = -e->nk; i <= e->nk; ++i)
        for (int j = -e->nk; j <= e->nk; ++j)
            for (int k = -e->nk; k <= e->nk; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                double k0 = g * i, k1 = g * j, k2 = g * k;
                double k2n = k0 * k0 + k1 * k1 + k2 * k2;
                if (k2n > e->kc * e->kc) continue;
                kadd(&s, &comp, exp(-k2n / (4.0 * e->alpha * e->alpha)) / k2n * cos(k0 * x[0] + k1 * x[1] + k2 * x[2]));
            }
    return 4.0 * M_PI / e->V * s;
}

static double ewald_psi(const ewald_par *e, const double x[3])
{
    return ewald_real(e, x, 0) + ewald_recip(e, x) - M_PI / (e->alpha * e->alpha * e->V);
}

double or_ewald_energy(int n, const double *xyz, const double *q, double a, double alpha,
                       double rc, double kc)
{
    ewald_par e = ewald_setup(a, alpha, rc, kc);
    double zero[3] = {0.0, 0.0, 0.0};
    double psi_self = ewald_real(&e, zero, 1) + ewald_recip(&e, zero) - 2.0 * alpha / sqrt(M_PI) -
                      M_PI / (alpha * alpha * e.V);
    double U = 0.0;
#pragma omp parallel for reduction(+ : U) schedule(dynamic, 4)
    for (int i = 0; i < n; ++i) {
        double ui = 0.5 * q[i] * q[i] * psi_self;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {xyz[3 * i] - xyz[3 * j], xyz[3 * i + 1] - xyz[3 * j + 1],
                           xyz[3 * i + 2] - xyz[3 * j + 2]};
            ui += 0.5 * q[i] * q[j] * ewald_psi(&e, d);
        }
        U += ui;
    }
    return U;
}

void or_ewald_dU(int n, const double *xyz, const double *q, double a, double alpha, double rc,
                 double kc, int np, const int64_t *idx, const double *tgt, double *dU)
{
    ewald_par e = ewald_setup(a, alpha, rc, kc);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < np; ++s) {
        int64_t i = idx[s];
        const double *t = tgt + 3 * s, *r = xyz + 3 * i;
        double acc = 0.0;
        int bad = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const double *rj = xyz + 3 * j;
            double dn[3] = {t[0] - rj[0], t[1] - rj[1], t[2] - rj[2]};
            double dold[3] = {r[0] - rj[0], r[1] - rj[1], r[2] - rj[2]};
            /* a target on another charge (or on one of its copies) is singular */
            double w[3];
            for (int c = 0; c < 3; ++c) w[c] = dn[c] - a * floor(dn[c] / a + 0.5);
            if (w[0] == 0.0 && w[1] == 0.0 && w[2] == 0.0) bad = 1;
            acc += q[j] * (ewald_psi(&e, dn) - ewald_psi(&e, dold));
        }
        dU[s] = bad ? NAN : q[i] * acc;
    }
}

/* parameters chosen like the Python helper ewald_params: rc = a/2 and both
 * truncations below 10^-16.5 */
static ewald_par self_change_params(double a)
{
    double x = 1.0;
    while (exp(-x * x) / x > pow(10.0, -16.5)) x += 0.01;
    double rc = 0.5 * a, alpha = x / rc;
    return ewald_setup(a, alpha, rc, 2.0 * alpha * x);
}

double or_periodic_self_change(double a, const double d[3])
{
    ewald_par e = self_change_params(a);
    double zero[3] = {0.0, 0.0, 0.0};
    double psi_self = ewald_real(&e, zero, 1) + ewald_recip(&e, zero) - 2.0 * e.alpha / sqrt(M_PI) -
                      M_PI / (e.alpha * e.alpha * e.V);
    /* reduce d to its nearest image: psi is periodic and the real-space sum
     * assumes |d_k| <= a/2 */
    double w[3];
    for (int k = 0; k < 3; ++k) w[k] = d[k] - a * floor(d[k] / a + 0.5);
    return psi_self - ewald_psi(&e, w);
}
