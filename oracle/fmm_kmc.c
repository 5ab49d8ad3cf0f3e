/*
 * O-fmm: the FMM-KMC method of the paper, step by step, in FP64.
 * Test infrastructure only: see oracle.h.
 *
 * Octree (Sec. 2.2): L levels, level l has 8^{l-1} cubic cells of side
 * a / 2^{l-1}; cell (ix,iy,iz) covers [ix w, (ix+1) w) x ...; a point's fine
 * cell is floor(x / w) per axis, capped at 2^{L-1} - 1.
 *
 * Setup (Alg. "fmm", App. A):
 *   P2M of the charges of every fine cell about its centre, M2M up to level 1.
 *   Downward pass, l = 2..L:  Psi_l = T_LL Psi_{l-1}(parent) + sum_{IL} T_ML Phi_l,
 *   IL(alpha) = children(N_b(parent(alpha))) \ (alpha u N_b(alpha)).
 *   Free space (Sec. 2.2.1): Psi_1 = Psi_2 = 0 (the interaction lists of levels
 *   1 and 2 are empty).  Periodic (Sec. 3.1, near-field component): Psi_1 = 0
 *   and Psi_2 starts from zero; interaction lists and neighbour lists are not
 *   truncated at the box but wrapped, a wrapped cell being the periodic copy of
 *   a primary cell at its geometric (shifted) position.  Psi_{L,alpha} then
 *   holds the field of every charge copy in the 3x3x3 block of boxes around the
 *   primary box except those in the 27 cells around alpha.
 *
 * Far field (Sec. 3.1): K_n^m = sum q r^n Y_n^{-m}, E_n^m = sum q r^n Y_n^m
 *   about the box centre, H = R K, with R the M2L operator whose geometric
 *   factor is the lattice sum over V_inf (lattice.c), plus the dipole term of
 *   Sec. 2.2.2 / App. B written into the degree-1 coefficients of H:
 *   H_1^k += -(4 pi / 3V) K_1^k, the local expansion of the compensating
 *   potential -(4 pi/3V) M.(x - c) in this normalisation.
 *
 * Proposal r -> r' of charge i (charge q, fine cell alpha, r' in cell alpha'):
 *   free space, Eq. (proposed_energy):
 *     dU = q (Psi_{alpha'}(r') + sum_{near(alpha')} q_j/|r'-r_j|)
 *        - q (Psi_alpha(r) + sum_{near(alpha), j != i} q_j/|r - r_j|) - q^2/|r'-r|
 *   periodic, Eq. (proposed_energy_sr) with r' wrapped into the box, plus
 *     dU_far = U_inf(r') - U_inf(r) with U_inf = 1/2 sum E H, evaluated as
 *     dE.H + 1/2 dE.(R dK) with dE = q(r'^n Y_n^m(r') - r^n Y_n^m(r)) and dK
 *     likewise with Y_n^{-m}.  This equals 1/2 (Ebar.Hbar - E.H) exactly
 *     because E.(R dK) = dE.(R K) (the copies nu and -nu are both in V_inf)
 *     and avoids subtracting two large numbers.  The factor 1/2 in U_inf is
 *     the same double-counting factor as in U_sr (reading of Sec. 3.1).
 *   With the exact self-image option (of_set_self_image) the V_box self terms,
 *   the constant and 1/2 dE.(R dK) are replaced by q^2 (psi_self - psi(r' - r)),
 *   psi the tin-foil Ewald pair potential (exact.c): the same quantity without
 *   truncation, so results move at truncation level.
 * Accept (Sec. 3, "Accept move"; Sec. 3.1): dU is recomputed (footnote of
 *   Sec. 3.1); every fine cell beta gets -P2L(q at r + a nu) for every copy nu
 *   (free space: nu = 0 only) that is not in the 27 cells around beta, and
 *   +P2L(q at r' + a nu) likewise; E += dE, K += dK, H = R K; U += dU.
 * Per-level expansions (the survey's next step f1: the O(log N) accept that the
 *   Introduction and Sec. 7 point to): Psi_l of level l holds only the M2L
 *   terms of its own interaction list, with no L2L from the parent, and the
 *   potential of a point is the sum over l = start..L of Psi_l of its level-l
 *   cell, each about that cell's centre (equal to the accumulated Psi_L up to
 *   rounding, since L2L of a truncated local expansion is exact).  The accept
 *   rule is then applied per level: Psi_{l,beta} gets -P2L(q at r + a nu) for
 *   every copy whose level-l cell lies in the interaction list of beta
 *   (outside the 27 cells around beta, inside the children of the 27 cells
 *   around its parent), and +P2L(q at r' + a nu) likewise, about the centre of
 *   beta.  This touches at most 189 cells per level and copy instead of every
 *   fine cell; the truncation differs from the fine-level rule, so results
 *   move at truncation level.
 * Uniform external field E (the applied field of Sec. 6.3): a proposal adds the
 *   work -q E.d done against it over the hop, d = r' - r (periodic: the minimum
 *   image); the total energy counts it through the accepted dU's.
 * Energy (Alg. "fmm_evaluation", with the charge q_i that the printed line 4
 *   leaves out): U = sum_i 1/2 q_i (Psi(r_i) + sum_{near, j != i} q_j / r_ij)
 *   + 1/2 sum E H.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "oracle_internal.h"

struct of_ctx {
    int bc, L, p, nt, n, lazy, start;
    double a;
    or_ops *ops;
    double *xyz, *q;
    int *cell;
    int **mem, *mcount, *mcap;
    cplx **phi;
    cplx **psi;
    char **psi_ok;
    int nlog, caplog;
    double *log_q, *log_old, *log_new;
    cplx *Gfar, *E, *K, *H;
    double U;
    int U_valid;
    int self_exact;
    int per_level; /* keep Psi_l of every level apart (no L2L) */
    double field[3]; /* uniform external field E */
};

static int side(int l) { return 1 << (l - 1); }
static int ncell(int l) { return side(l) * side(l) * side(l); }
static int cid(int n, int ix, int iy, int iz) { return (ix * n + iy) * n + iz; }
static void cxyz(int n, int c, int *ix, int *iy, int *iz)
{
    *iz = c % n;
    *iy = (c / n) % n;
    *ix = c / (n * n);
}
static int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }
static int posmod(int a, int b) { int r = a % b; return r < 0 ? r + b : r; }

static void centre(const of_ctx *c, int l, int ix, int iy, int iz, double out[3])
{
    double w = c->a / side(l);
    out[0] = (ix + 0.5) * w;
    out[1] = (iy + 0.5) * w;
    out[2] = (iz + 0.5) * w;
}

static void fine_index(const of_ctx *c, const double x[3], int g[3])
{
    int n = side(c->L);
    double w = c->a / n;
    for (int k = 0; k < 3; ++k) {
        int v = (int)floor(x[k] / w);
        if (v > n - 1) v = n - 1;
        if (v < 0) v = 0;
        g[k] = v;
    }
}

int of_fine_cell_of(of_ctx *c, const double x[3])
{
    int g[3];
    fine_index(c, x, g);
    return cid(side(c->L), g[0], g[1], g[2]);
}

static void member_add(of_ctx *c, int cell, int i)
{
    if (c->mcount[cell] == c->mcap[cell]) {
        c->mcap[cell] = c->mcap[cell] ? 2 * c->mcap[cell] : 4;
        c->mem[cell] = (int *)realloc(c->mem[cell], sizeof(int) * c->mcap[cell]);
    }
    c->mem[cell][c->mcount[cell]++] = i;
}

static void member_remove(of_ctx *c, int cell, int i)
{
    for (int k = 0; k < c->mcount[cell]; ++k)
        if (c->mem[cell][k] == i) {
            c->mem[cell][k] = c->mem[cell][--c->mcount[cell]];
            return;
        }
}

/* ---- setup -------------------------------------------------------------- */

static void upward(of_ctx *c, cplx **phi)
{
    int L = c->L, nt = c->nt, n = side(L);
#pragma omp parallel
    {
        cplx *Y = (cplx *)malloc(sizeof(cplx) * nt);
#pragma omp for schedule(dynamic, 16)
        for (int cc = 0; cc < ncell(L); ++cc) {
            int ix, iy, iz;
            cxyz(n, cc, &ix, &iy, &iz);
            double ctr[3];
            centre(c, L, ix, iy, iz, ctr);
            cplx *M = phi[L] + (size_t)cc * nt;
            memset(M, 0, sizeof(cplx) * nt);
            for (int k = 0; k < c->mcount[cc]; ++k) {
                int i = c->mem[cc][k];
                double d[3] = {c->xyz[3 * i] - ctr[0], c->xyz[3 * i + 1] - ctr[1], c->xyz[3 * i + 2] - ctr[2]};
                ops_p2m_add(c->ops, c->q[i], d, M, Y);
            }
        }
        free(Y);
    }
    for (int l = L - 1; l >= 1; --l) {
        int np = side(l), nc = side(l + 1);
#pragma omp parallel
        {
            cplx *Y = (cplx *)malloc(sizeof(cplx) * nt);
            cplx *T = (cplx *)malloc(sizeof(cplx) * nt);
#pragma omp for schedule(dynamic, 4)
            for (int pc = 0; pc < ncell(l); ++pc) {
                int px, py, pz;
                cxyz(np, pc, &px, &py, &pz);
                double pctr[3];
                centre(c, l, px, py, pz, pctr);
                cplx *M = phi[l] + (size_t)pc * nt;
                memset(M, 0, sizeof(cplx) * nt);
                for (int ch = 0; ch < 8; ++ch) {
                    int cx = 2 * px + (ch >> 2), cy = 2 * py + ((ch >> 1) & 1), cz = 2 * pz + (ch & 1);
                    double cctr[3];
                    centre(c, l + 1, cx, cy, cz, cctr);
                    double Q[3] = {cctr[0] - pctr[0], cctr[1] - pctr[1], cctr[2] - pctr[2]};
                    ops_m2m(c->ops, phi[l + 1] + (size_t)cid(nc, cx, cy, cz) * nt, Q, T, Y);
                    for (int k = 0; k < nt; ++k) M[k] += T[k];
                }
            }
            free(Y);
            free(T);
        }
    }
}

/* P2L update of one fine cell for one accepted move (the accept rule) */
static void accept_update_cell(of_ctx *c, int cell, double q, const double rold[3],
                               const double rnew[3], cplx *Y)
{
    int n = side(c->L), bx, by, bz;
    cxyz(n, cell, &bx, &by, &bz);
    double ctr[3];
    centre(c, c->L, bx, by, bz, ctr);
    int lim = c->bc ? 1 : 0;
    for (int e = 0; e < 2; ++e) {
        const double *y = e ? rnew : rold;
        double qq = e ? q : -q;
        int g0[3];
        fine_index(c, y, g0);
        for (int i = -lim; i <= lim; ++i)
            for (int j = -lim; j <= lim; ++j)
                for (int k = -lim; k <= lim; ++k) {
                    int g[3] = {g0[0] + i * n, g0[1] + j * n, g0[2] + k * n};
                    if (abs(g[0] - bx) <= 1 && abs(g[1] - by) <= 1 && abs(g[2] - bz) <= 1) continue;
                    double d[3] = {y[0] + c->a * i - ctr[0], y[1] + c->a * j - ctr[1], y[2] + c->a * k - ctr[2]};
                    ops_p2l_add(c->ops, qq, d, c->psi[c->L] + (size_t)cell * c->nt, Y);
                }
    }
}

/* per-level accept rule: P2L into cell `cell` of level l of every copy of the
 * two endpoints whose level-l cell is in the interaction list of `cell` */
static void accept_update_level(of_ctx *c, int l, int cell, double q, const double rold[3],
                                const double rnew[3], cplx *Y)
{
    int n = side(l), nf = side(c->L), bx, by, bz;
    cxyz(n, cell, &bx, &by, &bz);
    int b[3] = {bx, by, bz};
    double ctr[3];
    centre(c, l, bx, by, bz, ctr);
    int lim = c->bc ? 1 : 0, f = 1 << (c->L - l);
    for (int e = 0; e < 2; ++e) {
        const double *y = e ? rnew : rold;
        double qq = e ? q : -q;
        int g0[3];
        fine_index(c, y, g0);
        for (int i = -lim; i <= lim; ++i)
            for (int j = -lim; j <= lim; ++j)
                for (int k = -lim; k <= lim; ++k) {
                    int nu[3] = {i, j, k}, G[3], in_il = 0, near = 1, parent_near = 1;
                    for (int d = 0; d < 3; ++d) {
                        /* the copy's cell on level l, in unwrapped coordinates */
                        G[d] = floordiv(g0[d] + nu[d] * nf, f);
                        if (abs(G[d] - b[d]) > 1) near = 0;
                        if (abs(floordiv(G[d], 2) - floordiv(b[d], 2)) > 1) parent_near = 0;
                    }
                    in_il = !near && parent_near;
                    if (!in_il) continue;
                    double d[3] = {y[0] + c->a * i - ctr[0], y[1] + c->a * j - ctr[1], y[2] + c->a * k - ctr[2]};
                    ops_p2l_add(c->ops, qq, d, c->psi[l] + (size_t)cell * c->nt, Y);
                }
    }
}

/* Psi of one cell on level l, given Psi of its parent (if any) and Phi */
static void compute_psi(of_ctx *c, int l, int cell, cplx *Y, cplx *Y2)
{
    int nt = c->nt, n = side(l), ax, ay, az;
    cxyz(n, cell, &ax, &ay, &az);
    cplx *P = c->psi[l] + (size_t)cell * nt;
    memset(P, 0, sizeof(cplx) * nt);
    double ctr[3];
    centre(c, l, ax, ay, az, ctr);
    if (l - 1 >= c->start && !c->per_level) {
        int np = side(l - 1);
        int px = ax >> 1, py = ay >> 1, pz = az >> 1;
        double pctr[3];
        centre(c, l - 1, px, py, pz, pctr);
        double Q[3] = {pctr[0] - ctr[0], pctr[1] - ctr[1], pctr[2] - ctr[2]};
        ops_l2l_add(c->ops, c->psi[l - 1] + (size_t)cid(np, px, py, pz) * nt, Q, P, Y);
    }
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz) {
                if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) continue;
                int s[3] = {ax + dx, ay + dy, az + dz};
                if (abs(floordiv(s[0], 2) - (ax >> 1)) > 1 || abs(floordiv(s[1], 2) - (ay >> 1)) > 1 ||
                    abs(floordiv(s[2], 2) - (az >> 1)) > 1)
                    continue;
                int outside = 0;
                for (int k = 0; k < 3; ++k)
                    if (s[k] < 0 || s[k] >= n) outside = 1;
                if (outside && !c->bc) continue;
                int prim = cid(n, posmod(s[0], n), posmod(s[1], n), posmod(s[2], n));
                double sctr[3];
                centre(c, l, s[0], s[1], s[2], sctr); /* geometric centre of the copy */
                double Q[3] = {sctr[0] - ctr[0], sctr[1] - ctr[1], sctr[2] - ctr[2]};
                ops_m2l_add(c->ops, c->phi[l] + (size_t)prim * nt, Q, P, Y2);
            }
    if (c->per_level) {
        for (int e = 0; e < c->nlog; ++e)
            accept_update_level(c, l, cell, c->log_q[e], c->log_old + 3 * e, c->log_new + 3 * e, Y);
    } else if (l == c->L) {
        for (int e = 0; e < c->nlog; ++e)
            accept_update_cell(c, cell, c->log_q[e], c->log_old + 3 * e, c->log_new + 3 * e, Y);
    }
}

/* make sure Psi_L of the listed fine cells (and Psi of their ancestors) exist */
static void ensure_psi(of_ctx *c, int nreq, const int *req)
{
    int L = c->L;
    char *need = (char *)calloc(ncell(L), 1);
    for (int k = 0; k < nreq; ++k) need[req[k]] = 1;
    for (int l = c->start; l <= L; ++l) {
        int n = side(l), shift = L - l, nf = side(L);
        int *todo = (int *)malloc(sizeof(int) * ncell(l));
        char *mark = (char *)calloc(ncell(l), 1);
        int ntodo = 0;
        for (int f = 0; f < ncell(L); ++f) {
            if (!need[f]) continue;
            int fx, fy, fz;
            cxyz(nf, f, &fx, &fy, &fz);
            int cc = cid(n, fx >> shift, fy >> shift, fz >> shift);
            if (!c->psi_ok[l][cc] && !mark[cc]) {
                mark[cc] = 1;
                todo[ntodo++] = cc;
            }
        }
#pragma omp parallel
        {
            cplx *Y = (cplx *)malloc(sizeof(cplx) * c->nt);
            cplx *Y2 = (cplx *)malloc(sizeof(cplx) * (2 * c->p + 1) * (2 * c->p + 1));
#pragma omp for schedule(dynamic, 1)
            for (int t = 0; t < ntodo; ++t) compute_psi(c, l, todo[t], Y, Y2);
            free(Y);
            free(Y2);
        }
        for (int t = 0; t < ntodo; ++t) c->psi_ok[l][todo[t]] = 1;
        free(todo);
        free(mark);
    }
    free(need);
}

static void far_coefficients(const of_ctx *c, const double x[3], cplx *yp, cplx *ym, cplx *Y)
{
    /* x relative to the box centre: r^n Y_n^m and r^n Y_n^{-m} */
    double d[3] = {x[0] - 0.5 * c->a, x[1] - 0.5 * c->a, x[2] - 0.5 * c->a}, r, th, ph;
    or_spherical(d, &r, &th, &ph);
    or_sph_harmonics(c->p, th, ph, Y);
    double rn = 1.0;
    for (int n = 0; n <= c->p; ++n) {
        for (int m = -n; m <= n; ++m) {
            yp[or_idx(n, m)] = rn * Y[or_idx(n, m)];
            ym[or_idx(n, m)] = rn * Y[or_idx(n, -m)];
        }
        rn *= r;
    }
}

/* H = R K: lattice-sum M2L plus the dipole term */
static void apply_R(const of_ctx *c, const cplx *K, cplx *H)
{
    memset(H, 0, sizeof(cplx) * c->nt);
    ops_m2l_with_geometry(c->ops, K, c->Gfar, H);
    double V = c->a * c->a * c->a;
    for (int k = -1; k <= 1; ++k) H[or_idx(1, k)] += -(4.0 * M_PI / (3.0 * V)) * K[or_idx(1, k)];
}

of_ctx *of_create(int bc, double a, int L, int p, int n, const double *xyz, const double *q, int lazy)
{
    return of_create_levels(bc, a, L, p, n, xyz, q, lazy, 0);
}

of_ctx *of_create_levels(int bc, double a, int L, int p, int n, const double *xyz, const double *q, int lazy,
                         int per_level)
{
    of_ctx *c = (of_ctx *)calloc(1, sizeof(of_ctx));
    c->per_level = per_level ? 1 : 0;
    c->bc = bc;
    c->a = a;
    c->L = L;
    c->p = p;
    c->nt = (p + 1) * (p + 1);
    c->n = n;
    c->lazy = lazy;
    c->start = bc ? 2 : 3;
    c->ops = or_ops_create(p);
    c->xyz = (double *)malloc(sizeof(double) * 3 * n);
    c->q = (double *)malloc(sizeof(double) * n);
    memcpy(c->xyz, xyz, sizeof(double) * 3 * n);
    memcpy(c->q, q, sizeof(double) * n);
    c->cell = (int *)malloc(sizeof(int) * n);
    int nf = ncell(L);
    c->mem = (int **)calloc(nf, sizeof(int *));
    c->mcount = (int *)calloc(nf, sizeof(int));
    c->mcap = (int *)calloc(nf, sizeof(int));
    for (int i = 0; i < n; ++i) {
        c->cell[i] = of_fine_cell_of(c, xyz + 3 * i);
        member_add(c, c->cell[i], i);
    }
    c->phi = (cplx **)calloc(L + 1, sizeof(cplx *));
    c->psi = (cplx **)calloc(L + 1, sizeof(cplx *));
    c->psi_ok = (char **)calloc(L + 1, sizeof(char *));
    for (int l = 1; l <= L; ++l) {
        c->phi[l] = (cplx *)calloc((size_t)ncell(l) * c->nt, sizeof(cplx));
        c->psi[l] = (cplx *)calloc((size_t)ncell(l) * c->nt, sizeof(cplx));
        c->psi_ok[l] = (char *)calloc(ncell(l), 1);
    }
    upward(c, c->phi);
    if (!lazy) {
        int *all = (int *)malloc(sizeof(int) * nf);
        for (int k = 0; k < nf; ++k) all[k] = k;
        ensure_psi(c, nf, all);
        free(all);
    }
    if (bc) {
        int nt2 = (2 * p + 1) * (2 * p + 1);
        c->Gfar = (cplx *)malloc(sizeof(cplx) * nt2);
        or_lattice_sums(2 * p, c->Gfar);
        for (int s = 0; s <= 2 * p; ++s)
            for (int t = -s; t <= s; ++t) c->Gfar[or_idx(s, t)] *= pow(a, -(s + 1.0));
        c->E = (cplx *)calloc(c->nt, sizeof(cplx));
        c->K = (cplx *)calloc(c->nt, sizeof(cplx));
        c->H = (cplx *)calloc(c->nt, sizeof(cplx));
        cplx *yp = (cplx *)malloc(sizeof(cplx) * c->nt), *ym = (cplx *)malloc(sizeof(cplx) * c->nt),
             *Y = (cplx *)malloc(sizeof(cplx) * c->nt);
        for (int i = 0; i < n; ++i) {
            far_coefficients(c, xyz + 3 * i, yp, ym, Y);
            for (int k = 0; k < c->nt; ++k) {
                c->E[k] += q[i] * yp[k];
                c->K[k] += q[i] * ym[k];
            }
        }
        apply_R(c, c->K, c->H);
        free(yp);
        free(ym);
        free(Y);
    }
    /* energy, Alg. "fmm_evaluation" (+ far field); in lazy mode only on request,
     * since it needs the local expansion of every occupied cell */
    c->U = NAN;
    c->U_valid = 0;
    if (!lazy) of_energy(c);
    return c;
}

void of_set_self_image(of_ctx *c, int exact) { c->self_exact = exact ? 1 : 0; }

void of_set_field(of_ctx *c, const double E[3])
{
    for (int k = 0; k < 3; ++k) c->field[k] = E[k];
}

void of_destroy(of_ctx *c)
{
    if (!c) return;
    for (int l = 1; l <= c->L; ++l) {
        free(c->phi[l]);
        free(c->psi[l]);
        free(c->psi_ok[l]);
    }
    free(c->phi);
    free(c->psi);
    free(c->psi_ok);
    for (int k = 0; k < ncell(c->L); ++k) free(c->mem[k]);
    free(c->mem);
    free(c->mcount);
    free(c->mcap);
    free(c->xyz);
    free(c->q);
    free(c->cell);
    free(c->log_q);
    free(c->log_old);
    free(c->log_new);
    free(c->Gfar);
    free(c->E);
    free(c->K);
    free(c->H);
    or_ops_destroy(c->ops);
    free(c);
}

static void compute_energy(of_ctx *c)
{
    int n = c->n;
    int *req = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) req[i] = c->cell[i];
    ensure_psi(c, n, req);
    free(req);
    double U = 0.0;
#pragma omp parallel for reduction(+ : U) schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) U += 0.5 * c->q[i] * of_potential(c, c->xyz + 3 * i, i);
    /* of_potential includes the far-field potential: 1/2 sum q phi_inf = 1/2 E.H */
    c->U = U;
    c->U_valid = 1;
}

/* total energy; a lazy context computes the initial energy here if no move has
 * been accepted yet, and reports NaN otherwise */
double of_energy(of_ctx *c)
{
    if (!c->U_valid && c->nlog == 0) compute_energy(c);
    return c->U;
}
int of_nterms(of_ctx *c) { return c->nt; }

/* near-field sum at x over the 27 (wrapped) neighbour cells of fine cell g,
 * skipping charge `exclude` at its own (unshifted) position */
static double near_sum(const of_ctx *c, const double x[3], const int g[3], int64_t exclude)
{
    int n = side(c->L);
    double s = 0.0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int h[3] = {g[0] + dx, g[1] + dy, g[2] + dz};
                int outside = 0;
                for (int k = 0; k < 3; ++k)
                    if (h[k] < 0 || h[k] >= n) outside = 1;
                if (outside && !c->bc) continue;
                double sh[3];
                for (int k = 0; k < 3; ++k) sh[k] = c->a * floordiv(h[k], n);
                int prim = cid(n, posmod(h[0], n), posmod(h[1], n), posmod(h[2], n));
                for (int t = 0; t < c->mcount[prim]; ++t) {
                    int j = c->mem[prim][t];
                    if (j == exclude && sh[0] == 0.0 && sh[1] == 0.0 && sh[2] == 0.0) continue;
                    double d0 = x[0] - (c->xyz[3 * j] + sh[0]), d1 = x[1] - (c->xyz[3 * j + 1] + sh[1]),
                           d2 = x[2] - (c->xyz[3 * j + 2] + sh[2]);
                    s += c->q[j] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                }
            }
    return s;
}

/* the local-expansion part of the potential at x in fine cell g: Psi_L of the
 * cell, or with per-level expansions the sum over levels of Psi_l of the
 * level-l cell containing it, each about that cell's centre */
static double local_part(const of_ctx *c, const double x[3], const int g[3], cplx *Y)
{
    if (!c->per_level) {
        double ctr[3];
        centre(c, c->L, g[0], g[1], g[2], ctr);
        double d[3] = {x[0] - ctr[0], x[1] - ctr[1], x[2] - ctr[2]};
        return ops_eval_local(c->ops, c->psi[c->L] + (size_t)cid(side(c->L), g[0], g[1], g[2]) * c->nt, d, Y);
    }
    double s = 0.0;
    for (int l = c->start; l <= c->L; ++l) {
        int sh = c->L - l, ax = g[0] >> sh, ay = g[1] >> sh, az = g[2] >> sh;
        double ctr[3];
        centre(c, l, ax, ay, az, ctr);
        double d[3] = {x[0] - ctr[0], x[1] - ctr[1], x[2] - ctr[2]};
        s += ops_eval_local(c->ops, c->psi[l] + (size_t)cid(side(l), ax, ay, az) * c->nt, d, Y);
    }
    return s;
}

/* potential at x (a point of the box) from all charges except `exclude`;
 * Psi_L of x's cell must exist */
double of_potential(of_ctx *c, const double x[3], int64_t exclude)
{
    int g[3];
    fine_index(c, x, g);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * c->nt);
    double phi = local_part(c, x, g, Y);
    phi += near_sum(c, x, g, exclude);
    if (c->bc) {
        double e[3] = {x[0] - 0.5 * c->a, x[1] - 0.5 * c->a, x[2] - 0.5 * c->a};
        phi += ops_eval_local(c->ops, c->H, e, Y);
    }
    free(Y);
    return phi;
}

static int wrap_target(const of_ctx *c, const double t[3], double tw[3])
{
    for (int k = 0; k < 3; ++k) {
        if (c->bc) {
            tw[k] = t[k] - c->a * floor(t[k] / c->a);
            if (tw[k] >= c->a) tw[k] -= c->a;
        } else {
            if (!(t[k] >= 0.0 && t[k] < c->a)) return 0;
            tw[k] = t[k];
        }
    }
    return 1;
}

static int occupied(const of_ctx *c, const double x[3])
{
    int cell = of_fine_cell_of((of_ctx *)c, x);
    for (int t = 0; t < c->mcount[cell]; ++t) {
        int j = c->mem[cell][t];
        if (c->xyz[3 * j] == x[0] && c->xyz[3 * j + 1] == x[1] && c->xyz[3 * j + 2] == x[2]) return 1;
    }
    return 0;
}

/* dU of one proposal; Psi_L of the two cells must exist */
static double propose_one(of_ctx *c, int64_t i, const double t[3])
{
    double tw[3];
    if (!wrap_target(c, t, tw)) return NAN;
    if (occupied(c, tw)) return NAN;
    const double *r = c->xyz + 3 * i;
    double q = c->q[i];
    int ga[3], gb[3];
    fine_index(c, r, ga);
    fine_index(c, tw, gb);
    cplx *Y = (cplx *)malloc(sizeof(cplx) * c->nt);
    double phi_new = local_part(c, tw, gb, Y) + near_sum(c, tw, gb, -1);
    double phi_old = local_part(c, r, ga, Y) + near_sum(c, r, ga, i);
    double dU = q * phi_new - q * phi_old;
    if (!c->bc) {
        double d0 = tw[0] - r[0], d1 = tw[1] - r[1], d2 = tw[2] - r[2];
        dU -= q * q / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        dU -= q * (c->field[0] * d0 + c->field[1] * d1 + c->field[2] * d2);
        free(Y);
        return dU;
    }
    /* uniform field: the work -q E.d over the hop, d the minimum-image displacement */
    {
        double d[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = tw[k] - r[k];
            d[k] -= c->a * floor(d[k] / c->a + 0.5);
        }
        dU -= q * (c->field[0] * d[0] + c->field[1] * d[1] + c->field[2] * d[2]);
    }
    /* periodic: self terms of Eq. (proposed_energy_sr) */
    if (c->self_exact) {
        /* the exact change of the moving charge's interaction with its own copies */
        double d[3] = {tw[0] - r[0], tw[1] - r[1], tw[2] - r[2]};
        dU += q * q * or_periodic_self_change(c->a, d);
    } else {
        double self = 0.0;
        for (int a0 = -1; a0 <= 1; ++a0)
            for (int a1 = -1; a1 <= 1; ++a1)
                for (int a2 = -1; a2 <= 1; ++a2) {
                    double d0 = tw[0] - (r[0] + c->a * a0), d1 = tw[1] - (r[1] + c->a * a1),
                           d2 = tw[2] - (r[2] + c->a * a2);
                    self += 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                }
        dU += -q * q * self + q * q * (6.0 + 8.0 / sqrt(3.0) + 12.0 / sqrt(2.0)) / c->a;
    }
    /* far field */
    int nt = c->nt;
    cplx *ypn = (cplx *)malloc(sizeof(cplx) * nt), *ymn = (cplx *)malloc(sizeof(cplx) * nt);
    cplx *ypo = (cplx *)malloc(sizeof(cplx) * nt), *ymo = (cplx *)malloc(sizeof(cplx) * nt);
    cplx *dE = (cplx *)malloc(sizeof(cplx) * nt), *dK = (cplx *)malloc(sizeof(cplx) * nt);
    cplx *dH = (cplx *)malloc(sizeof(cplx) * nt);
    far_coefficients(c, tw, ypn, ymn, Y);
    far_coefficients(c, r, ypo, ymo, Y);
    for (int k = 0; k < nt; ++k) {
        dE[k] = q * (ypn[k] - ypo[k]);
        dK[k] = q * (ymn[k] - ymo[k]);
    }
    apply_R(c, dK, dH);
    cplx s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < nt; ++k) {
        s1 += dE[k] * c->H[k];
        s2 += dE[k] * dH[k];
    }
    /* with the exact self term, 1/2 dE.R'dK (the copies in V_inf of the moving
     * charge seen from its new place) is already part of it */
    dU += creal(s1) + (c->self_exact ? 0.0 : 0.5 * creal(s2));
    free(ypn);
    free(ymn);
    free(ypo);
    free(ymo);
    free(dE);
    free(dK);
    free(dH);
    free(Y);
    return dU;
}

void of_propose(of_ctx *c, int np, const int64_t *idx, const double *tgt, double *dU)
{
    int *req = (int *)malloc(sizeof(int) * 2 * (size_t)np);
    int nreq = 0;
    for (int s = 0; s < np; ++s) {
        req[nreq++] = c->cell[idx[s]];
        double tw[3];
        if (wrap_target(c, tgt + 3 * s, tw)) req[nreq++] = of_fine_cell_of(c, tw);
    }
    ensure_psi(c, nreq, req);
    free(req);
#pragma omp parallel for schedule(dynamic, 16)
    for (int s = 0; s < np; ++s) dU[s] = propose_one(c, idx[s], tgt + 3 * s);
}

double of_accept(of_ctx *c, int64_t i, const double newpos[3])
{
    double dU;
    of_propose(c, 1, &i, newpos, &dU);
    if (isnan(dU)) return NAN;
    double tw[3];
    wrap_target(c, newpos, tw);
    double rold[3] = {c->xyz[3 * i], c->xyz[3 * i + 1], c->xyz[3 * i + 2]};
    double q = c->q[i];
    /* fine-level local expansions of the cells that exist (all of them unless lazy) */
    int L = c->L, nf = ncell(L);
#pragma omp parallel
    {
        cplx *Y = (cplx *)malloc(sizeof(cplx) * c->nt);
#pragma omp for schedule(dynamic, 16)
        for (int b = 0; b < nf; ++b)
            if (c->psi_ok[L][b] && !c->per_level) accept_update_cell(c, b, q, rold, tw, Y);
        free(Y);
    }
    if (c->per_level) {
        for (int l = c->start; l <= L; ++l) {
#pragma omp parallel
            {
                cplx *Y = (cplx *)malloc(sizeof(cplx) * c->nt);
#pragma omp for schedule(dynamic, 16)
                for (int b = 0; b < ncell(l); ++b)
                    if (c->psi_ok[l][b]) accept_update_level(c, l, b, q, rold, tw, Y);
                free(Y);
            }
        }
    }
    /* log for cells whose local expansion is formed later */
    if (c->nlog == c->caplog) {
        c->caplog = c->caplog ? 2 * c->caplog : 64;
        c->log_q = (double *)realloc(c->log_q, sizeof(double) * c->caplog);
        c->log_old = (double *)realloc(c->log_old, sizeof(double) * 3 * c->caplog);
        c->log_new = (double *)realloc(c->log_new, sizeof(double) * 3 * c->caplog);
    }
    c->log_q[c->nlog] = q;
    memcpy(c->log_old + 3 * c->nlog, rold, sizeof(rold));
    memcpy(c->log_new + 3 * c->nlog, tw, sizeof(tw));
    c->nlog++;
    if (c->bc) {
        int nt = c->nt;
        cplx *ypn = (cplx *)malloc(sizeof(cplx) * nt), *ymn = (cplx *)malloc(sizeof(cplx) * nt);
        cplx *ypo = (cplx *)malloc(sizeof(cplx) * nt), *ymo = (cplx *)malloc(sizeof(cplx) * nt);
        cplx *Y = (cplx *)malloc(sizeof(cplx) * nt);
        far_coefficients(c, tw, ypn, ymn, Y);
        far_coefficients(c, rold, ypo, ymo, Y);
        for (int k = 0; k < nt; ++k) {
            c->E[k] += q * (ypn[k] - ypo[k]);
            c->K[k] += q * (ymn[k] - ymo[k]);
        }
        apply_R(c, c->K, c->H);
        free(ypn);
        free(ymn);
        free(ypo);
        free(ymo);
        free(Y);
    }
    member_remove(c, c->cell[i], (int)i);
    memcpy(c->xyz + 3 * i, tw, sizeof(tw));
    c->cell[i] = of_fine_cell_of(c, tw);
    member_add(c, c->cell[i], (int)i);
    c->U += dU;
    return dU;
}

void of_get_local(of_ctx *c, int cell, cplx *out)
{
    ensure_psi(c, 1, &cell);
    memcpy(out, c->psi[c->L] + (size_t)cell * c->nt, sizeof(cplx) * c->nt);
}

/* Psi of one cell on level l (formed first if needed) */
void of_get_level_local(of_ctx *c, int level, int cell, cplx *out)
{
    int sh = c->L - level, n = side(level), nf = side(c->L);
    int ax, ay, az;
    cxyz(n, cell, &ax, &ay, &az);
    int fine = cid(nf, ax << sh, ay << sh, az << sh);
    ensure_psi(c, 1, &fine);
    memcpy(out, c->psi[level] + (size_t)cell * c->nt, sizeof(cplx) * c->nt);
}

void of_get_multipole(of_ctx *c, int level, int cell, cplx *out)
{
    memcpy(out, c->phi[level] + (size_t)cell * c->nt, sizeof(cplx) * c->nt);
}

void of_get_far(of_ctx *c, cplx *E, cplx *K, cplx *H)
{
    if (!c->bc) return;
    memcpy(E, c->E, sizeof(cplx) * c->nt);
    memcpy(K, c->K, sizeof(cplx) * c->nt);
    memcpy(H, c->H, sizeof(cplx) * c->nt);
}

void of_get_positions(of_ctx *c, double *xyz) { memcpy(xyz, c->xyz, sizeof(double) * 3 * c->n); }

/* multipole expansion of one cell for the current positions (a fresh upward
 * pass; used to check an incrementally maintained tree) */
void of_rebuild_multipoles(of_ctx *c, int level, int cell, cplx *out)
{
    cplx **phi = (cplx **)calloc(c->L + 1, sizeof(cplx *));
    for (int l = 1; l <= c->L; ++l) phi[l] = (cplx *)calloc((size_t)ncell(l) * c->nt, sizeof(cplx));
    upward(c, phi);
    memcpy(out, phi[level] + (size_t)cell * c->nt, sizeof(cplx) * c->nt);
    for (int l = 1; l <= c->L; ++l) free(phi[l]);
    free(phi);
}
