// Accept-step kernels (Sec. 3 "Accept move", Sec. 3.1 "Accept move").
//
// Sweep: every fine cell beta gets -P2L(q at r + a nu) for every copy nu of the
// old position (free space: nu = 0 only; periodic: the 27 copies in V_box) whose
// cell is not one of the 27 cells around beta, and +P2L(q at r' + a nu)
// likewise.  P2L of a point charge is the multipole-to-local translation of a
// monopole, L_n^m = q I_n^m(y - c_beta).  One lane per (cell, order m): the lane
// runs the irregular recurrence down column m and owns coefficients (n, m),
// n >= m, of its cell, so no two lanes write the same word.
//
// Path: the multipole expansions of the old and new cell of the moved charge
// on every level change by -/+ its P2M; level 1 is the box multipole K of the
// far field.
#include "kernels.hpp"

namespace fmmkmc {

struct Move {
    double ox, oy, oz;   // old position (in the box)
    double nx, ny, nz;   // new position (in the box)
    double q;
    int ogx, ogy, ogz;   // fine-cell coordinates of the old position
    int ngx, ngy, ngz;   // and of the new one
};

template <int P, int Mc>
__device__ void sweep_column(const Geo g, int64_t M, int64_t cell, const Move mv, double *__restrict__ psi,
                             float *__restrict__ psi32)
{
    constexpr int NC = P - Mc + 1;
    double accr[NC], acci[NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) accr[t] = acci[t] = 0.0;
    const int nc = g.nc;
    const int bx = (int)(cell / ((int64_t)nc * nc)), by = (int)((cell / nc) % nc), bz = (int)(cell % nc);
    const double cxw = (bx + 0.5) * g.w, cyw = (by + 0.5) * g.w, czw = (bz + 0.5) * g.w;
    const int lim = g.periodic ? 1 : 0;
    for (int e = 0; e < 2; ++e) {
        const double px = e ? mv.nx : mv.ox, py = e ? mv.ny : mv.oy, pz = e ? mv.nz : mv.oz;
        const int gx0 = e ? mv.ngx : mv.ogx, gy0 = e ? mv.ngy : mv.ogy, gz0 = e ? mv.ngz : mv.ogz;
        const double qq = e ? mv.q : -mv.q;
        for (int i = -lim; i <= lim; ++i)
            for (int j = -lim; j <= lim; ++j)
                for (int k = -lim; k <= lim; ++k) {
                    const int gx = gx0 + i * nc, gy = gy0 + j * nc, gz = gz0 + k * nc;
                    if (abs(gx - bx) <= 1 && abs(gy - by) <= 1 && abs(gz - bz) <= 1) continue;
                    const double dx = px + g.a * i - cxw, dy = py + g.a * j - cyw, dz = pz + g.a * k - czw;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double ir2 = 1.0 / r2;
                    double dr = 1.0 / sqrt(r2), di = 0.0;
#pragma unroll
                    for (int m = 1; m <= Mc; ++m) {
                        const double f = -(2 * m - 1) * ir2;
                        double ndr = f * (dx * dr - dy * di), ndi = f * (dx * di + dy * dr);
                        dr = ndr;
                        di = ndi;
                    }
                    double ar = dr, ai = di;
                    accr[0] += qq * ar;
                    acci[0] += qq * ai;
                    double br = (2 * Mc + 1) * dz * ir2 * ar, bi = (2 * Mc + 1) * dz * ir2 * ai;
                    if (NC > 1) {
                        accr[1] += qq * br;
                        acci[1] += qq * bi;
                    }
#pragma unroll
                    for (int t = 2; t < NC; ++t) {
                        const int n = Mc + t;
                        const double cf = (double)((n - 1) * (n - 1) - Mc * Mc);
                        double cr = ((2 * n - 1) * dz * br - cf * ar) * ir2;
                        double ci = ((2 * n - 1) * dz * bi - cf * ai) * ir2;
                        accr[t] += qq * cr;
                        acci[t] += qq * ci;
                        ar = br;
                        ai = bi;
                        br = cr;
                        bi = ci;
                    }
                }
    }
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        const int n = Mc + t;
        if (Mc == 0) {
            const int64_t at = (int64_t)slot0(n) * M + cell;
            const double v = psi[at] + accr[t];
            psi[at] = v;
            if (psi32) psi32[at] = (float)v;
        } else {
            const int64_t ar_ = (int64_t)slot_re(n, Mc) * M + cell, ai_ = (int64_t)slot_im(n, Mc) * M + cell;
            const double vr = psi[ar_] + accr[t], vi = psi[ai_] + acci[t];
            psi[ar_] = vr;
            psi[ai_] = vi;
            if (psi32) {
                psi32[ar_] = (float)vr;
                psi32[ai_] = (float)vi;
            }
        }
    }
}

template <int P, int Mc = 0>
__device__ void sweep_dispatch(int m, const Geo g, int64_t M, int64_t cell, const Move &mv, double *psi,
                               float *psi32)
{
    if constexpr (Mc <= P) {
        if (m == Mc)
            sweep_column<P, Mc>(g, M, cell, mv, psi, psi32);
        else
            sweep_dispatch<P, Mc + 1>(m, g, M, cell, mv, psi, psi32);
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_sweep(Geo g, int64_t M, Move mv, double *__restrict__ psi,
                                               float *__restrict__ psi32)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= M) return;
    sweep_dispatch<P>(blockIdx.y, g, M, cell, mv, psi, psi32);
}

// P2M of -q at the old and +q at the new position into the cells containing
// them on every level; one lane per (level, m), both endpoints in turn.
__global__ void k_path(Geo g, int L, int p, Move mv, double *const *__restrict__ phi)
{
    const int t = threadIdx.x;
    if (t >= L * (p + 1)) return;
    const int l = 1 + t / (p + 1), m = t % (p + 1);
    const int nl = 1 << (l - 1), sh = (L - l);
    const double w = g.a / nl;
    const int64_t Ml = (int64_t)nl * nl * nl;
    double *ph = phi[l];
    for (int e = 0; e < 2; ++e) {
        const double px = e ? mv.nx : mv.ox, py = e ? mv.ny : mv.oy, pz = e ? mv.nz : mv.oz;
        const int gx = (e ? mv.ngx : mv.ogx) >> sh, gy = (e ? mv.ngy : mv.ogy) >> sh, gz = (e ? mv.ngz : mv.ogz) >> sh;
        const double qq = e ? mv.q : -mv.q;
        const int64_t cell = cell_id(nl, gx, gy, gz);
        const double dx = px - (gx + 0.5) * w, dy = py - (gy + 0.5) * w, dz = pz - (gz + 0.5) * w;
        const double r2 = dx * dx + dy * dy + dz * dz;
        double dr = 1.0, di = 0.0;
        for (int k = 1; k <= m; ++k) {
            const double f = -0.5 / k;
            double ndr = f * (dx * dr - dy * di), ndi = f * (dx * di + dy * dr);
            dr = ndr;
            di = ndi;
        }
        double ar = dr, ai = di, br = 0, bi = 0;
        for (int n = m; n <= p; ++n) {
            double cr, ci;
            if (n == m) {
                cr = ar;
                ci = ai;
            } else if (n == m + 1) {
                cr = dz * ar;
                ci = dz * ai;
                br = cr;
                bi = ci;
            } else {
                const double wgt = rinv(n, m);
                cr = ((2 * n - 1) * dz * br - r2 * ar) * wgt;
                ci = ((2 * n - 1) * dz * bi - r2 * ai) * wgt;
                ar = br;
                ai = bi;
                br = cr;
                bi = ci;
            }
            if (m == 0) {
                ph[(int64_t)slot0(n) * Ml + cell] += qq * cr;
            } else {
                ph[(int64_t)slot_re(n, m) * Ml + cell] += qq * cr;
                ph[(int64_t)slot_im(n, m) * Ml + cell] -= qq * ci;
            }
        }
    }
}

// position, cell-slot and site bookkeeping of the moved charge
struct Book {
    int64_t i;
    double nx, ny, nz, q;
    int64_t old_cell, new_cell;
    int old_slot, new_slot;
    int moved_j;          // charge moved into old_slot (-1 if none)
    int old_cnt, new_cnt; // counts after the move
    int64_t old_site, new_site;        // lattice order, -1 if no lattice
    int64_t old_site_s2, new_site_s2;  // cell-major (2x2x2 path), -1 if unused
    int same_cell;        // the move stays inside one fine cell: slots unchanged
};

__global__ void k_book(Book b, double *x, double *y, double *z, int32_t *cell, int32_t *slot, int32_t *site,
                       int32_t *cnt, int32_t *slots, int cap, int32_t *site_charge, double *qsite, float *qsite32)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    x[b.i] = b.nx;
    y[b.i] = b.ny;
    z[b.i] = b.nz;
    if (!b.same_cell) {
        // old cell: the last slot's charge fills the hole (old_cnt < cap after removal)
        if (b.moved_j >= 0) {
            slots[b.old_cell * cap + b.old_slot] = b.moved_j;
            slot[b.moved_j] = b.old_slot;
        }
        slots[b.old_cell * cap + b.old_cnt] = -1;
        cnt[b.old_cell] = b.old_cnt;
        slots[b.new_cell * cap + b.new_slot] = (int32_t)b.i;
        cnt[b.new_cell] = b.new_cnt;
        cell[b.i] = (int32_t)b.new_cell;
        slot[b.i] = b.new_slot;
    }
    if (b.old_site >= 0) {
        site_charge[b.old_site] = -1;
        site_charge[b.new_site] = (int32_t)b.i;
        site[b.i] = (int32_t)b.new_site;
    }
    if (b.old_site_s2 >= 0) {
        qsite[b.old_site_s2] = 0.0;
        qsite[b.new_site_s2] = b.q;
        if (qsite32) {
            qsite32[b.old_site_s2] = 0.0f;
            qsite32[b.new_site_s2] = (float)b.q;
        }
    }
}

void launch_commit(fmmkmc_ctx *c, const Geo &g, const CommitArgs &a)
{
    Move mv;
    mv.ox = a.old_pos[0];
    mv.oy = a.old_pos[1];
    mv.oz = a.old_pos[2];
    mv.nx = a.new_pos[0];
    mv.ny = a.new_pos[1];
    mv.nz = a.new_pos[2];
    mv.q = a.q;
    mv.ogx = a.old_g[0];
    mv.ogy = a.old_g[1];
    mv.ogz = a.old_g[2];
    mv.ngx = a.new_g[0];
    mv.ngy = a.new_g[1];
    mv.ngz = a.new_g[2];
    dim3 grid((unsigned)((c->M + 255) / 256), c->p + 1);
    float *p32 = c->prec == FMMKMC_MIXED ? c->psi32 : nullptr;
    FMMKMC_DISPATCH_P(c->p, launch(c, "sweep", k_sweep<P_>, grid, dim3(256), g, c->M, mv, c->psi_lv[c->L], p32));
    launch(c, "path", k_path, dim3(1), dim3(kMaxLevels * (kMaxOrder + 1)), g, c->L, c->p, mv, c->d_phi_ptrs);
    Book b;
    b.i = a.i;
    b.nx = a.new_pos[0];
    b.ny = a.new_pos[1];
    b.nz = a.new_pos[2];
    b.q = a.q;
    b.old_cell = a.old_cell;
    b.new_cell = a.new_cell;
    b.old_slot = a.old_slot;
    b.new_slot = a.new_slot;
    b.moved_j = a.moved_j;
    b.old_cnt = a.old_cnt;
    b.new_cnt = a.new_cnt;
    b.old_site = a.old_site;
    b.new_site = a.new_site;
    b.old_site_s2 = c->s2 ? a.old_site_s2 : -1;
    b.new_site_s2 = c->s2 ? a.new_site_s2 : -1;
    b.same_cell = a.old_cell == a.new_cell ? 1 : 0;
    launch(c, "book", k_book, dim3(1), dim3(64), b, c->x, c->y, c->z, c->cell, c->slot, c->site, c->cell_cnt,
           c->cell_slots, c->cap, c->site_charge, c->qsite, c->qsite32);
}

}  // namespace fmmkmc
