// Accept-step kernels (Sec. 3 "Accept move", Sec. 3.1 "Accept move").
//
// Sweep: every fine cell beta gets -P2L(q at r + a nu) for every copy nu of the
// old position (free space: nu = 0 only; periodic: the 27 copies in V_box) whose
// cell is not one of the 27 cells around beta, and +P2L(q at r' + a nu)
// likewise.  P2L of a point charge is the multipole-to-local translation of a
// monopole, L_n^m = q I_n^m(y - c_beta).  One lane per (cell, group of orders
// m): the lane runs the irregular recurrences down its columns and owns
// coefficients (n, m), n >= m, of its cell, so no two lanes write the same word.
//
// Per-level expansions (see fmmkmc_params.per_level): the same P2L, applied on
// every level l to the cells beta of that level whose interaction list holds
// the copy (its level-l cell outside the 27 around beta, inside the children
// of the 27 around beta's parent).  Such cells lie within 3 cells of the copy,
// so a commit visits the 7^3 blocks around the two endpoints on each level.
//
// Path: the multipole expansions of the old and new cell of the moved charge
// on every level change by -/+ its P2M; level 1 is the box multipole K of the
// far field.
#include "batch.hpp"
#include "kernels.hpp"

namespace fmmkmc {


// Columns m of the local expansion are split into groups whose coefficients
// fit in registers (at most sweep_budget(P) doubles); one lane per (cell,
// group).  The per-source work (offset, 1/r, the near test) is shared by a
// group's columns, and the irregular diagonal I_m^m is carried across them, so
// fewer groups repeat that work less often; 59 doubles give three groups at
// p = 12 (four at 56) within 168 VGPRs, i.e. three waves per SIMD, which the
// sweep needs to hide its FP64 dependency chains (two groups at p = 10 would
// need 65 and spill).
__host__ __device__ constexpr int sweep_budget(int) { return 59; }
__host__ __device__ constexpr int col_cost(int P, int m) { return m == 0 ? P + 1 : 2 * (P - m + 1); }
__host__ __device__ constexpr int group_end(int P, int m0)
{
    int acc = col_cost(P, m0), m = m0;
    while (m + 1 <= P && acc + col_cost(P, m + 1) <= sweep_budget(P)) acc += col_cost(P, ++m);
    return m;
}
__host__ __device__ constexpr int n_groups(int P)
{
    int g = 0, m = 0;
    while (m <= P) {
        m = group_end(P, m) + 1;
        ++g;
    }
    return g;
}
__host__ __device__ constexpr int group_m0(int P, int g)
{
    int m = 0;
    for (int i = 0; i < g; ++i) m = group_end(P, m) + 1;
    return m;
}
__host__ __device__ constexpr int col_offset(int P, int M0, int m)
{
    int o = 0;
    for (int t = M0; t < m; ++t) o += col_cost(P, t);
    return o;
}

// 1/sqrt(x) for x > 0: the hardware estimate (about 24 correct bits on
// gfx950, measured) refined by one Newton-Raphson step y <- y (3 - x y^2) / 2,
// which doubles the correct bits: within 20 ulp over 1e-6..1e6 (a second step
// reaches 1.6 ulp), far below what the expansions are truncated at.
__device__ inline double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    return y;
}

// Scaled irregular harmonics.  With rho = 1/|d| and the unit vector
// (xh, yh, zh) = rho d, write I_n^m(d) = q rho^(n+1) (2n-1)!! T_n^m; the
// recurrences of I become
//   T_0^0 = 1,  T_m^m = -(xh + i yh) T_{m-1}^{m-1},  T_{m+1}^m = zh T_m^m,
//   T_n^m = zh T_{n-1}^m - c_n^m T_{n-2}^m,  c_n^m = ((n-1)^2 - m^2) / ((2n-1)(2n-3)),
// with constant coefficients.  The columns are carried rescaled once more,
// U_n^m = T_n^m / s_n^m with s_m = s_{m+1} = 1 and s_n = c_n^m s_{n-2}, which
// turns the three-term step into U_n = (g_n^m zh) U_{n-1} - U_{n-2} with
// g_n^m = s_{n-1} / s_n: one multiply shared by the real and imaginary parts
// and one fused multiply-add each.  The accumulation is one fused multiply-add
// with q rho^(n+1); (2n-1)!! s_n^m is applied once per cell when the sums are
// added to the expansion.
template <int P>
struct ScaledIrregular {
    double g[P + 1][P + 1];      // s_{n-1} / s_n for n >= m + 2
    double scale[P + 1][P + 1];  // (2n-1)!! s_n^m
    constexpr ScaledIrregular() : g{}, scale{}
    {
        for (int m = 0; m <= P; ++m) {
            double s2 = 1.0, s1 = 1.0;  // s_{n-2}, s_{n-1}
            double f = 1.0;
            for (int n = 1; n <= m; ++n) f *= (double)(2 * n - 1);
            for (int n = m; n <= P; ++n) {
                if (n > m) f *= (double)(2 * n - 1);
                double sn = 1.0;
                if (n >= m + 2) {
                    const double c = (double)((n - 1) * (n - 1) - m * m) / (double)((2 * n - 1) * (2 * n - 3));
                    sn = c * s2;
                    g[n][m] = s1 / sn;
                }
                scale[n][m] = f * sn;
                if (n >= m + 1) {
                    s2 = s1;
                    s1 = sn;
                } else {
                    s1 = sn;
                }
            }
        }
    }
};

// The sources of a move: -q at the old and +q at the new position, each with
// its copies nu in V_box (periodic; 2 x 27) or alone (free space; 2).  Every
// lane of a block reads the same source at the same time, so the block builds
// this table once in LDS: the copy's position, its charge and its fine-cell
// coordinates (unwrapped, for the near-field test).  mnear: whether the copy
// can lie in the near field of any of the block's cells (its cell within one
// of the bounding box of the block's cells); for all other copies the lanes
// skip their own near-field test.
struct SweepSources {
    double x[54], y[54], z[54], q[54];
    int gx[54], gy[54], gz[54];
    int mnear[54];
};

// by the first 2 x 27 (2) threads of the block; a barrier must follow.  The
// block's fine cells are c0 .. c1 (cell order); c1 < c0: unknown (every copy
// is marked as possibly near).
__device__ inline void sweep_sources(const Geo &g, const Move &mv, SweepSources &S, int64_t c0 = 0, int64_t c1 = -1)
{
    const int nimg = g.periodic ? 27 : 1;
    const int t = threadIdx.x;
    if (t < 2 * nimg) {
        const int e = t >= nimg ? 1 : 0;
        const int nu = t - e * nimg;
        const int i = g.periodic ? nu / 9 - 1 : 0, j = g.periodic ? (nu / 3) % 3 - 1 : 0,
                  k = g.periodic ? nu % 3 - 1 : 0;
        S.gx[t] = (e ? mv.ngx : mv.ogx) + i * g.nc;
        S.gy[t] = (e ? mv.ngy : mv.ogy) + j * g.nc;
        S.gz[t] = (e ? mv.ngz : mv.ogz) + k * g.nc;
        S.x[t] = (e ? mv.nx : mv.ox) + g.a * i;
        S.y[t] = (e ? mv.ny : mv.oy) + g.a * j;
        S.z[t] = (e ? mv.nz : mv.oz) + g.a * k;
        S.q[t] = e ? mv.q : -mv.q;
        int mn = 1;
        if (c1 >= c0) {
            // bounding box of the cells c0 .. c1: consecutive cell ids share x
            // (then y) only if the first and the last one do
            const int nc = g.nc;
            const int x0 = (int)(c0 / ((int64_t)nc * nc)), y0 = (int)((c0 / nc) % nc), z0 = (int)(c0 % nc);
            const int x1 = (int)(c1 / ((int64_t)nc * nc)), y1 = (int)((c1 / nc) % nc), z1 = (int)(c1 % nc);
            const bool sx = x0 == x1, sxy = sx && y0 == y1;
            const int by0 = sx ? y0 : 0, by1 = sx ? y1 : nc - 1, bz0 = sxy ? z0 : 0, bz1 = sxy ? z1 : nc - 1;
            mn = S.gx[t] >= x0 - 1 && S.gx[t] <= x1 + 1 && S.gy[t] >= by0 - 1 && S.gy[t] <= by1 + 1 &&
                 S.gz[t] >= bz0 - 1 && S.gz[t] <= bz1 + 1;
        }
        S.mnear[t] = mn;
    }
}

// PD, PF: pointers to the FP64 expansions and their FP32 shadow (or null),
// generic or global-space.  LEVEL: g is the geometry of a coarser level whose
// cells are the fine cells shifted right by sh, and a copy contributes only
// from the interaction list (the per-level rule); else every copy outside the
// near field contributes.
template <int P, int M0, int M1, bool LEVEL, class PD, class PF>
__device__ void sweep_cols(const Geo g, int64_t M, int64_t cell, const SweepSources &S, uint64_t mmask, PD psi,
                           PF psi32, int sh)
{
    constexpr ScaledIrregular<P> SI{};
    constexpr int NACC = col_offset(P, M0, M1 + 1);
    double acc[NACC];
#pragma unroll
    for (int t = 0; t < NACC; ++t) acc[t] = 0.0;
    const int nc = g.nc;
    const int bx = (int)(cell / ((int64_t)nc * nc)), by = (int)((cell / nc) % nc), bz = (int)(cell % nc);
    const double cxw = (bx + 0.5) * g.w, cyw = (by + 0.5) * g.w, czw = (bz + 0.5) * g.w;
    // a source copy whose cell is one of the 27 around this cell is in the
    // near field and contributes with charge 0 (no branch, so the sums stay in
    // place across iterations)
    const int nsrc = g.periodic ? 54 : 2;
#pragma unroll 1
    for (int t = 0; t < nsrc; ++t) {
        // a copy that no cell of the block has in its near field skips the
        // per-lane test (a block-uniform branch; the sums are the same)
        const bool mn = LEVEL || ((mmask >> t) & 1);
        bool near = false;
        if (mn) {
            int sx = S.gx[t], sy = S.gy[t], sz = S.gz[t];
            if (LEVEL) {  // arithmetic shifts: floor division of the unwrapped coordinates
                sx >>= sh;
                sy >>= sh;
                sz >>= sh;
            }
            near = ((unsigned)(sx - bx + 1) <= 2u) & ((unsigned)(sy - by + 1) <= 2u) & ((unsigned)(sz - bz + 1) <= 2u);
            if (LEVEL) {
                const bool parent_near = ((unsigned)((sx >> 1) - (bx >> 1) + 1) <= 2u) &
                                         ((unsigned)((sy >> 1) - (by >> 1) + 1) <= 2u) &
                                         ((unsigned)((sz >> 1) - (bz >> 1) + 1) <= 2u);
                near = near | !parent_near;  // outside the interaction list: no contribution
                // most copies lie in no target's interaction list on the finer levels:
                // skip a copy that no lane of the wave takes (a wave-uniform branch)
                if (!__any(!near)) continue;
            }
        }
        // for a near copy the weights are exactly zero; 1/|d| is taken as 1 so
        // that every factor stays finite (|d| may be 0), and the zero weights
        // then add exactly nothing
        const double dx = S.x[t] - cxw, dy = S.y[t] - cyw, dz = S.z[t] - czw;
        const double qq = near ? 0.0 : S.q[t];
        const double rho = rsqrt_nr(near ? 1.0 : dx * dx + dy * dy + dz * dz);
        const double xh = dx * rho, yh = dy * rho, zh = dz * rho;
        double w[P + 1];  // q rho^(n+1)
        w[0] = qq * rho;
#pragma unroll
        for (int n = 1; n <= P; ++n) w[n] = w[n - 1] * rho;
        // diagonal T_m^m = z^m with z = -(xh + i yh): the group's first order
        // M0 by repeated squaring, then one step per order
        double dr = 1.0, di = 0.0;
        {
            double br = -xh, bi = -yh;  // z^(2^b)
#pragma unroll
            for (int b = 0; (1 << b) <= M0; ++b) {
                if ((M0 >> b) & 1) {
                    if ((M0 & ((1 << b) - 1)) == 0) {  // the lowest set bit: z^(2^b) itself
                        dr = br;
                        di = bi;
                    } else {
                        const double ndr = dr * br - di * bi, ndi = dr * bi + di * br;
                        dr = ndr;
                        di = ndi;
                    }
                }
                if ((2 << b) <= M0) {
                    const double nbr = br * br - bi * bi, nbi = 2.0 * br * bi;
                    br = nbr;
                    bi = nbi;
                }
            }
        }
#pragma unroll
        for (int m = M0; m <= M1; ++m) {
            if (m > M0) {
                const double ndr = yh * di - xh * dr, ndi = -(xh * di + yh * dr);
                dr = ndr;
                di = ndi;
            }
            {
                const int o = col_offset(P, M0, m);
                const bool cplxcol = m > 0;
                double ar = dr, ai = di;
                acc[o] = fma(w[m], ar, acc[o]);
                if (cplxcol) acc[o + 1] = fma(w[m], ai, acc[o + 1]);
                if (m + 1 <= P) {
                    double br = zh * ar, bi = zh * ai;
                    acc[o + (cplxcol ? 2 : 1)] = fma(w[m + 1], br, acc[o + (cplxcol ? 2 : 1)]);
                    if (cplxcol) acc[o + 3] = fma(w[m + 1], bi, acc[o + 3]);
#pragma unroll
                    for (int n = m + 2; n <= P; ++n) {
                        const double gz = zh * SI.g[n][m];
                        const double cr = fma(gz, br, -ar), ci = fma(gz, bi, -ai);
                        const int tt = n - m;
                        acc[o + (cplxcol ? 2 * tt : tt)] = fma(w[n], cr, acc[o + (cplxcol ? 2 * tt : tt)]);
                        if (cplxcol) acc[o + 2 * tt + 1] = fma(w[n], ci, acc[o + 2 * tt + 1]);
                        ar = br;
                        ai = bi;
                        br = cr;
                        bi = ci;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int m = M0; m <= M1; ++m) {
        const int o = col_offset(P, M0, m);
#pragma unroll
        for (int n = m; n <= P; ++n) {
            const int t = n - m;
            const double f = SI.scale[n][m];
            if (m == 0) {
                const int64_t at = (int64_t)slot0(n) * M + cell;
                const double v = fma(f, acc[o + t], psi[at]);
                psi[at] = v;
                if (psi32) psi32[at] = (float)v;
            } else {
                const int64_t ar_ = (int64_t)slot_re(n, m) * M + cell, ai_ = (int64_t)slot_im(n, m) * M + cell;
                const double vr = fma(f, acc[o + 2 * t], psi[ar_]), vi = fma(f, acc[o + 2 * t + 1], psi[ai_]);
                psi[ar_] = vr;
                psi[ai_] = vi;
                if (psi32) {
                    psi32[ar_] = (float)vr;
                    psi32[ai_] = (float)vi;
                }
            }
        }
    }
}

// mmask: bit t set if source copy t may lie in the near field of a cell of the
// block (sweep_near_mask); LEVEL ignores it
template <int P, bool LEVEL = false, int G = 0, class PD, class PF>
__device__ void sweep_dispatch(int grp, const Geo g, int64_t M, int64_t cell, const SweepSources &S, uint64_t mmask,
                               PD psi, PF psi32, int sh = 0)
{
    if constexpr (G < n_groups(P)) {
        if (grp == G)
            sweep_cols<P, group_m0(P, G), group_end(P, group_m0(P, G)), LEVEL>(g, M, cell, S, mmask, psi, psi32,
                                                                             sh);
        else
            sweep_dispatch<P, LEVEL, G + 1>(grp, g, M, cell, S, mmask, psi, psi32, sh);
    }
}

// the copies' mnear flags as a wave-uniform bit mask; every lane of the wave
// must take part (before any lane leaves)
__device__ inline uint64_t sweep_near_mask(const Geo &g, const SweepSources &S)
{
    const int lane = (int)(threadIdx.x & 63);
    return __ballot(lane < (g.periodic ? 54 : 2) && S.mnear[lane] != 0);
}

// Target t of a per-level commit: level lstart + t / (2 * 343), then the 7^3
// block around the old (first) or new (second) endpoint's cell on that level.
// A level with at most 7 cells per axis is enumerated once, cell by cell; the
// new endpoint's block skips the cells of the old one's, so no cell is visited
// twice and no two lanes write the same expansion.
__device__ inline bool level_target(const Geo &g, const Move &mv, int64_t t, int &level, int64_t &cell)
{
    const int per = 2 * 343;
    const int li = (int)(t / per);
    if (li > g.L - g.lstart) return false;
    level = g.lstart + li;
    const int rem = (int)(t - (int64_t)li * per), e = rem / 343, d = rem % 343;
    const int side = 1 << (level - 1), sh = g.L - level;
    if (side <= 7) {
        if (e == 1 || d >= side * side * side) return false;
        cell = d;
        return true;
    }
    const int ox = mv.ogx >> sh, oy = mv.ogy >> sh, oz = mv.ogz >> sh;
    int bx = (e ? mv.ngx >> sh : ox) + d / 49 - 3, by = (e ? mv.ngy >> sh : oy) + (d / 7) % 7 - 3,
        bz = (e ? mv.ngz >> sh : oz) + d % 7 - 3;
    if (g.periodic) {
        bx = posmod(bx, side);
        by = posmod(by, side);
        bz = posmod(bz, side);
    } else if (bx < 0 || bx >= side || by < 0 || by >= side || bz < 0 || bz >= side) {
        return false;
    }
    if (e == 1) {
        auto dist = [&](int u, int v) {
            if (!g.periodic) return abs(u - v);
            const int w = posmod(u - v, side);
            return w < side - w ? w : side - w;
        };
        if (dist(bx, ox) <= 3 && dist(by, oy) <= 3 && dist(bz, oz) <= 3) return false;
    }
    cell = cell_id(side, bx, by, bz);
    return true;
}

__host__ __device__ inline int64_t level_targets(int L, int lstart) { return (int64_t)(L - lstart + 1) * 2 * 343; }

// the per-level commit of one target (level, cell) and one column group
template <int P, class PD, class PF>
__device__ inline void levels_body(int grp, const Geo &gf, const Move &mv, const SweepSources &S, int64_t t,
                                   PD const *psi_lv, PF psi32)
{
    int level;
    int64_t cell;
    if (!level_target(gf, mv, t, level, cell)) return;
    Geo g = gf;
    g.nc = 1 << (level - 1);
    g.w = gf.a / g.nc;
    const int64_t Ml = (int64_t)g.nc * g.nc * g.nc;
    sweep_dispatch<P, true>(grp, g, Ml, cell, S, ~0ull, psi_lv[level], level == gf.L ? psi32 : (PF) nullptr,
                            gf.L - level);
}

template <int P>
__global__ __launch_bounds__(256) void k_levels(Geo g, Move mv, double *const *__restrict__ psi_lv,
                                                float *__restrict__ psi32)
{
    __shared__ SweepSources S;
    sweep_sources(g, mv, S);
    __syncthreads();
    levels_body<P>(blockIdx.y, g, mv, S, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, psi_lv, psi32);
}

template <int P>
__global__ __launch_bounds__(256, 3) void k_sweep(Geo g, int64_t M, Move mv, double *__restrict__ psi,
                                               float *__restrict__ psi32)
{
    __shared__ SweepSources S;
    const int64_t c0 = (int64_t)blockIdx.x * blockDim.x;
    sweep_sources(g, mv, S, c0, (c0 + blockDim.x < M ? c0 + blockDim.x : M) - 1);
    __syncthreads();
    const uint64_t mmask = sweep_near_mask(g, S);
    const int64_t cell = c0 + threadIdx.x;
    if (cell >= M) return;
    sweep_dispatch<P>(blockIdx.y, g, M, cell, S, mmask, psi, psi32);
}

// P2M of -q at the old and +q at the new position into the cells containing
// them on every level; one lane per (level, n, m >= 0) runs the regular
// recurrence to R_n^m itself, for both endpoints in turn.
__device__ __forceinline__ void path_body(int64_t blk, Geo g, int L, int p, const Move &mv,
                                          double *const *__restrict__ phi)
{
    const int per = (p + 1) * (p + 2) / 2;
    const int t = (int)(blk * blockDim.x + threadIdx.x);
    if (t >= L * per) return;
    const int l = 1 + t / per;
    int r = t % per, n = 0;
    while (r > n) {
        r -= n + 1;
        ++n;
    }
    const int m = r;
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
            const double ndr = f * (dx * dr - dy * di), ndi = f * (dx * di + dy * dr);
            dr = ndr;
            di = ndi;
        }
        double ar = dr, ai = di, br = dz * dr, bi = dz * di;
        double cr = ar, ci = ai;
        if (n == m + 1) {
            cr = br;
            ci = bi;
        }
        for (int k = m + 2; k <= n; ++k) {
            const double wgt = rinv(k, m);
            cr = ((2 * k - 1) * dz * br - r2 * ar) * wgt;
            ci = ((2 * k - 1) * dz * bi - r2 * ai) * wgt;
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

__global__ void k_path(Geo g, int L, int p, Move mv, double *const *__restrict__ phi)
{
    path_body(blockIdx.x, g, L, p, mv, phi);
}

// position, cell-slot and site bookkeeping of the moved charge

__device__ __forceinline__ void book_body(const Book &b, double *x, double *y, double *z, int32_t *cell,
                                          int32_t *slot, int32_t *site, int32_t *ijk_r, int32_t *cnt,
                                          int32_t *slots, int cap, int32_t *site_charge, int32_t *site_rank,
                                          double *qsite, float *qsite32)
{
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
    if (b.new_site >= 0) {
        site_charge[b.old_sord] = -1;
        site_charge[b.new_sord] = (int32_t)b.i;
        site_rank[b.old_sord] = -1;
        site_rank[b.new_sord] = b.rank;
        site[b.i] = (int32_t)b.new_site;
        ijk_r[b.rank] = b.new_ijk;
        if (qsite) {
            qsite[b.old_sord] = 0.0;
            qsite[b.new_sord] = b.q;
            if (qsite32) {
                qsite32[b.old_sord] = 0.0f;
                qsite32[b.new_sord] = (float)b.q;
            }
        }
    }
}

__global__ void k_book(Book b, double *x, double *y, double *z, int32_t *cell, int32_t *slot, int32_t *site,
                       int32_t *ijk_r, int32_t *cnt, int32_t *slots, int cap, int32_t *site_charge,
                       int32_t *site_rank, double *qsite, float *qsite32)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    book_body(b, x, y, z, cell, slot, site, ijk_r, cnt, slots, cap, site_charge, site_rank, qsite, qsite32);
}

void launch_commit(fmmkmc_ctx *c, const Geo &g, const CommitArgs &a, hipStream_t side)
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
    float *p32 = c->prec == FMMKMC_MIXED ? c->psi32 : nullptr;
    if (c->per_level) {
        const int64_t nt_ = level_targets(g.L, g.lstart);
        FMMKMC_DISPATCH_P(c->p, launch(c, "levels", k_levels<P_>, dim3((unsigned)((nt_ + 255) / 256), n_groups(P_)),
                                       dim3(256), g, mv, (double *const *)c->d_psi_ptrs, p32));
    } else {
        FMMKMC_DISPATCH_P(c->p, launch(c, "sweep", k_sweep<P_>, dim3((unsigned)((c->M + 255) / 256), n_groups(P_)),
                                       dim3(256), g, c->M, mv, c->psi_lv[c->L], p32));
    }
    const int per = (c->p + 1) * (c->p + 2) / 2;
    launch_on(c, side, "path", k_path, dim3((c->L * per + 255) / 256), dim3(256), 0, g, c->L, c->p, mv,
              c->d_phi_ptrs);
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
    b.new_site = a.new_site;
    b.old_sord = a.old_sord;
    b.new_sord = a.new_sord;
    b.new_ijk = a.new_ijk;
    b.rank = a.rank;
    b.s2 = c->s2 ? 1 : 0;
    b.same_cell = a.old_cell == a.new_cell ? 1 : 0;
    launch_on(c, side, "book", k_book, dim3(1), dim3(64), 0, b, c->x, c->y, c->z, c->cell, c->slot, c->site,
              c->ijk_r, c->cell_cnt, c->cell_slots, c->cap, c->site_charge, c->site_rank, c->qsite, c->qsite32);
}


// ---- batched replicas ---------------------------------------------------------

template <int P>
__global__ __launch_bounds__(256, 3) void k_b_sweep(const RepDev *__restrict__ reps, int R,
                                                 const int64_t *__restrict__ base, const MoveDev *__restrict__ moves)
{
    const int r = find_rep(base, R, blockIdx.x);
    const MoveDev &mv = moves[r];
    if (!mv.valid) return;  // uniform over the block
    const RepDev &d = reps[r];
    __shared__ SweepSources S;
    const int64_t c0 = (blockIdx.x - base[r]) * blockDim.x;
    sweep_sources(d.g, mv.mv, S, c0, (c0 + blockDim.x < d.M ? c0 + blockDim.x : d.M) - 1);
    __syncthreads();
    const uint64_t mmask = sweep_near_mask(d.g, S);
    const int64_t cell = c0 + threadIdx.x;
    if (cell >= d.M) return;
    // The expansions' pointers come from the replica table, so the compiler
    // cannot tell they address global memory and would use flat loads and
    // stores for the write-back; global-space pointers keep it global.
    using GD = __attribute__((address_space(1))) double;
    using GF = __attribute__((address_space(1))) float;
    sweep_dispatch<P>(blockIdx.y, d.g, d.M, cell, S, mmask, (GD *)d.psi, (GF *)d.psi32);
}

// per-level commit of every replica: nb blocks per replica
template <int P>
__global__ __launch_bounds__(256) void k_b_levels(const RepDev *__restrict__ reps, const MoveDev *__restrict__ moves,
                                                  int nb)
{
    const int r = blockIdx.x / nb;
    const MoveDev &mv = moves[r];
    if (!mv.valid) return;  // uniform over the block
    const RepDev &d = reps[r];
    __shared__ SweepSources S;
    sweep_sources(d.g, mv.mv, S);
    __syncthreads();
    using GD = __attribute__((address_space(1))) double;
    using GF = __attribute__((address_space(1))) float;
    levels_body<P>(blockIdx.y, d.g, mv.mv, S, (int64_t)(blockIdx.x % nb) * blockDim.x + threadIdx.x,
                   (GD *const *)d.psi_lv, (GF *)d.psi32);
}

void launch_b_levels(Profiler &pr, hipStream_t st, const RepDev *reps, int R, int p, const MoveDev *moves, int Lmax,
                     int lstart)
{
    const int nb = (int)((level_targets(Lmax, lstart) + 255) / 256);
    FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_levels", k_b_levels<P_>, dim3((unsigned)(R * nb), n_groups(P_)),
                                     dim3(256), 0, reps, moves, nb));
}

__global__ void k_b_path(const RepDev *__restrict__ reps, int R, const int64_t *__restrict__ base,
                         const MoveDev *__restrict__ moves)
{
    const int r = find_rep(base, R, blockIdx.x);
    const MoveDev &mv = moves[r];
    if (!mv.valid) return;
    const RepDev &d = reps[r];
    path_body(blockIdx.x - base[r], d.g, d.L, d.p, mv.mv, d.phi_lv);
}

// one lane per replica
__global__ void k_b_book(const RepDev *__restrict__ reps, int R, const MoveDev *__restrict__ moves)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R || !moves[r].valid) return;
    const RepDev &d = reps[r];
    book_body(moves[r].bk, d.x, d.y, d.z, d.cell, d.slot, d.site, d.ijk_r, d.cnt, d.slots, d.cap, d.site_charge,
              d.site_rank, d.qsite, d.qsite32);
}

void launch_b_sweep(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                    int p, const MoveDev *moves, int block)
{
    if (block < 64) block = 64;  // the block fills its 54-entry source table with one thread per entry
    FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_sweep", k_b_sweep<P_>, dim3((unsigned)blocks, n_groups(P_)),
                                     dim3(block), 0, reps, R, base, moves));
}

void launch_b_path(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                   const MoveDev *moves)
{
    launch_prof(pr, st, "b_path", k_b_path, dim3((unsigned)blocks), dim3(256), 0, reps, R, base, moves);
}

void launch_b_book(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const MoveDev *moves)
{
    launch_prof(pr, st, "b_book", k_b_book, dim3((unsigned)((R + 63) / 64)), dim3(64), 0, reps, R, moves);
}

}  // namespace fmmkmc
