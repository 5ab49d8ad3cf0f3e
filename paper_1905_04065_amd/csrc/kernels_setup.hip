// Setup kernels: Alg. "fmm" (App. A) of the paper on the GPU.
//   P2M   multipole of the charges of each fine cell about its centre
//   M2M   upward pass, child -> parent (8 fixed child offsets per level)
//   M2L + L2L downward pass per level: Psi = T_LL Psi(parent) + sum_{IL} T_ML Phi
//         (free space: levels 1-2 have empty interaction lists, Sec. 2.2.1;
//          periodic: Psi_1 = 0 and wrapped interaction lists from level 2, Sec. 3.1)
//   far   H = R K of the periodic copies in V_inf (Sec. 3.1) and its Chebyshev
//         form for fast evaluation at lattice sites.
// Expansions are stored coefficient-major, [k][cell], so a wavefront of
// consecutive cells reads each coefficient row with one coalesced access.
#include "batch.hpp"
#include "kernels.hpp"

namespace fmmkmc {

// ---- P2M: one lane per (fine cell, order m) -------------------------------

template <int P, int Mc>
__device__ void p2m_column(const Geo g, int64_t M, int64_t cell, const double *__restrict__ x,
                           const double *__restrict__ y, const double *__restrict__ z,
                           const double *__restrict__ q, const int32_t *__restrict__ cnt,
                           const int32_t *__restrict__ slots, double *__restrict__ phi)
{
    constexpr int NC = P - Mc + 1;
    double accr[NC], acci[NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) accr[t] = acci[t] = 0.0;
    const int cx = (int)(cell / ((int64_t)g.nc * g.nc)), cy = (int)((cell / g.nc) % g.nc), cz = (int)(cell % g.nc);
    const double ox = (cx + 0.5) * g.w, oy = (cy + 0.5) * g.w, oz = (cz + 0.5) * g.w;
    const int c = cnt[cell];
    for (int s = 0; s < c; ++s) {
        const int j = slots[cell * g.cap + s];
        const double dx = x[j] - ox, dy = y[j] - oy, dz = z[j] - oz, qq = q[j];
        const double r2 = dx * dx + dy * dy + dz * dz;
        double dr = 1.0, di = 0.0;
#pragma unroll
        for (int m = 1; m <= Mc; ++m) {
            const double f = -0.5 / m;
            double ndr = f * (dx * dr - dy * di), ndi = f * (dx * di + dy * dr);
            dr = ndr;
            di = ndi;
        }
        double ar = dr, ai = di, br = dz * dr, bi = dz * di;
        accr[0] += qq * ar;
        acci[0] -= qq * ai;
        if (NC > 1) {
            accr[1] += qq * br;
            acci[1] -= qq * bi;
        }
#pragma unroll
        for (int t = 2; t < NC; ++t) {
            const int n = Mc + t;
            const double w = rinv(n, Mc);
            double cr = ((2 * n - 1) * dz * br - r2 * ar) * w;
            double ci = ((2 * n - 1) * dz * bi - r2 * ai) * w;
            accr[t] += qq * cr;
            acci[t] -= qq * ci;
            ar = br;
            ai = bi;
            br = cr;
            bi = ci;
        }
    }
#pragma unroll
    for (int t = 0; t < NC; ++t) {
        const int n = Mc + t;
        if (Mc == 0) {
            phi[(int64_t)slot0(n) * M + cell] = accr[t];
        } else {
            phi[(int64_t)slot_re(n, Mc) * M + cell] = accr[t];
            phi[(int64_t)slot_im(n, Mc) * M + cell] = acci[t];
        }
    }
}

template <int P, int Mc = 0>
__device__ void p2m_dispatch(int m, const Geo g, int64_t M, int64_t cell, const double *x, const double *y,
                             const double *z, const double *q, const int32_t *cnt, const int32_t *slots,
                             double *phi)
{
    if constexpr (Mc <= P) {
        if (m == Mc)
            p2m_column<P, Mc>(g, M, cell, x, y, z, q, cnt, slots, phi);
        else
            p2m_dispatch<P, Mc + 1>(m, g, M, cell, x, y, z, q, cnt, slots, phi);
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_p2m(Geo g, int64_t M, const double *__restrict__ x,
                                             const double *__restrict__ y, const double *__restrict__ z,
                                             const double *__restrict__ q, const int32_t *__restrict__ cnt,
                                             const int32_t *__restrict__ slots, double *__restrict__ phi)
{
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= M) return;
    p2m_dispatch<P>(blockIdx.y, g, M, cell, x, y, z, q, cnt, slots, phi);
}

void launch_p2m(fmmkmc_ctx *c, const Geo &g)
{
    dim3 grid((unsigned)((c->M + 255) / 256), c->p + 1);
    FMMKMC_DISPATCH_P(c->p, launch(c, "p2m", k_p2m<P_>, grid, dim3(256), g, c->M, c->x, c->y, c->z, c->q,
                                   c->cell_cnt, c->cell_slots, c->phi_lv[c->L]));
}

// ---- matrix-vector translation kernels ------------------------------------
// out[k][cell] = sum_n mat[n][k] * in[n][cell'] with in/out rows coalesced over
// consecutive cells.

// matrix entries a thread loads at once before using them (the sums still run
// in order of n)
constexpr int kPre = 16;

// M2M: one thread per (parent cell, output coefficient k).  The threads of a
// wave share the parent (each parent takes nt rounded up to a multiple of 64
// threads), so they read the same child coefficients and consecutive matrix
// entries; the sum runs over the 8 children, then n.
__global__ __launch_bounds__(256) void k_m2m(int nt, int ncp, const double *__restrict__ mats,
                                             const double *__restrict__ child, double *__restrict__ parent)
{
    const int64_t Mp = (int64_t)ncp * ncp * ncp, Mc = Mp * 8;
    const int ncc = 2 * ncp;
    const int KP = (nt + 63) & ~63;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t pc = gt / KP;
    const int k = (int)(gt - pc * KP);
    if (pc >= Mp || k >= nt) return;
    const int px = (int)(pc / ((int64_t)ncp * ncp)), py = (int)((pc / ncp) % ncp), pz = (int)(pc % ncp);
    double acc = 0.0;
    for (int ch = 0; ch < 8; ++ch) {
        const int64_t cc = cell_id(ncc, 2 * px + (ch >> 2), 2 * py + ((ch >> 1) & 1), 2 * pz + (ch & 1));
        const double *col = mats + (int64_t)ch * nt * nt + k;
        const double *cv = child + cc;
        int n = 0;
        for (; n + kPre <= nt; n += kPre) {
            double mv[kPre], xv[kPre];
#pragma unroll
            for (int j = 0; j < kPre; ++j) {
                mv[j] = col[(int64_t)(n + j) * nt];
                xv[j] = cv[(int64_t)(n + j) * Mc];
            }
#pragma unroll
            for (int j = 0; j < kPre; ++j) acc += mv[j] * xv[j];
        }
        for (; n < nt; ++n) acc += col[(int64_t)n * nt] * cv[(int64_t)n * Mc];
    }
    parent[(int64_t)k * Mp + pc] = acc;
}

int64_t m2m_blocks(int nt, int ncp)
{
    const int64_t threads = (int64_t)ncp * ncp * ncp * ((nt + 63) & ~63);
    return (threads + 255) / 256;
}

// acc[c] += sum_n mat[n][k] * stage[n][c] over n in order, the column entries
// loaded kPre at a time
template <int C>
__device__ __forceinline__ void column_times_stage(double (&acc)[C], const double *__restrict__ mat, int k, int nt,
                                                   const double *stage)
{
    const double *col = mat + k;
    int n = 0;
    for (; n + kPre <= nt; n += kPre) {
        double tv[kPre];
#pragma unroll
        for (int j = 0; j < kPre; ++j) tv[j] = col[(int64_t)(n + j) * nt];
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const double *sr = stage + (n + j) * C;
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] += tv[j] * sr[c];
        }
    }
    for (; n < nt; ++n) {
        const double tv = col[(int64_t)n * nt];
        const double *sr = stage + n * C;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += tv * sr[c];
    }
}

// M2L + L2L for one level.  A block takes C target cells of one parity class
// (the position of a cell within its parent), which share the 189
// interaction-list offsets, and one thread per output coefficient k (KPT per
// thread when (p+1)^2 > 256).  For each offset the source coefficients of the
// C cells are staged in LDS (scaled by w^-deg(n): the M2L matrices are for unit
// cell width), and a thread runs down its column of the matrix with coalesced
// loads, using each staged coefficient C times; outputs get w^-(deg(k)+1), the
// parent's local expansion is added through the L2L matrix of the parity
// class, and the block writes its C x (p+1)^2 results through LDS.
template <int C, int KPT>
__global__ __launch_bounds__(256) void k_m2l(int nt, int nc, int periodic, int with_parent,
                                             const double *__restrict__ m2l, const int32_t *__restrict__ m2l_index,
                                             const double *__restrict__ scale_in, const double *__restrict__ scale_out,
                                             const double *__restrict__ l2l, const double *__restrict__ phi,
                                             const double *__restrict__ psi_parent, double *__restrict__ psi)
{
    extern __shared__ double stage[];  // [nt][C]
    const int pcls = blockIdx.y;
    const int px = pcls >> 2, py = (pcls >> 1) & 1, pz = pcls & 1;
    const int h = nc / 2;
    const int64_t Mh = (int64_t)h * h * h, M = Mh * 8;
    const int64_t t0 = (int64_t)blockIdx.x * C;
    const int ncell = (int)(Mh - t0 < C ? Mh - t0 : C);
    double acc[KPT][C];
#pragma unroll
    for (int u = 0; u < KPT; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[u][c] = 0.0;
    for (int dx = -2 - px; dx <= 3 - px; ++dx)
        for (int dy = -2 - py; dy <= 3 - py; ++dy)
            for (int dz = -2 - pz; dz <= 3 - pz; ++dz) {
                if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
                for (int e = threadIdx.x; e < nt * C; e += blockDim.x) {
                    const int n = e / C, c = e - n * C;
                    double v = 0.0;
                    if (c < ncell) {
                        const int64_t t = t0 + c;
                        const int ix = (int)(t / ((int64_t)h * h)), iy = (int)((t / h) % h), iz = (int)(t % h);
                        int sx = 2 * ix + px + dx, sy = 2 * iy + py + dy, sz = 2 * iz + pz + dz;
                        const bool outside = sx < 0 || sx >= nc || sy < 0 || sy >= nc || sz < 0 || sz >= nc;
                        if (!outside || periodic) {
                            sx = posmod(sx, nc);
                            sy = posmod(sy, nc);
                            sz = posmod(sz, nc);
                            v = phi[(int64_t)n * M + cell_id(nc, sx, sy, sz)] * scale_in[n];
                        }
                    }
                    stage[e] = v;
                }
                __syncthreads();
                // the matrix converts a source at offset -d to the target: d = target - source
                const double *mat = m2l + (int64_t)m2l_index[(-dx + 3) * 49 + (-dy + 3) * 7 + (-dz + 3)] * nt * nt;
#pragma unroll
                for (int u = 0; u < KPT; ++u) {
                    const int k = threadIdx.x + u * 256;
                    if (k < nt) column_times_stage<C>(acc[u], mat, k, nt, stage);
                }
                __syncthreads();
            }
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
        const int k = threadIdx.x + u * 256;
        const double so = k < nt ? scale_out[k] : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) acc[u][c] *= so;
    }
    if (with_parent) {
        for (int e = threadIdx.x; e < nt * C; e += blockDim.x) {
            const int n = e / C, c = e - n * C;
            double v = 0.0;
            if (c < ncell) v = psi_parent[(int64_t)n * Mh + t0 + c];  // parent index = class index
            stage[e] = v;
        }
        __syncthreads();
        const double *mat = l2l + (int64_t)pcls * nt * nt;
#pragma unroll
        for (int u = 0; u < KPT; ++u) {
            const int k = threadIdx.x + u * 256;
            if (k < nt) column_times_stage<C>(acc[u], mat, k, nt, stage);
        }
        __syncthreads();
    }
    // results through LDS: [k][c], then coalesced over the block's cells
    for (int u = 0; u < KPT; ++u) {
        const int k = threadIdx.x + u * 256;
        if (k < nt)
#pragma unroll
            for (int c = 0; c < C; ++c) stage[k * C + c] = acc[u][c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nt * C; e += blockDim.x) {
        const int k = e / C, c = e - k * C;
        if (c >= ncell) continue;
        const int64_t t = t0 + c;
        const int ix = (int)(t / ((int64_t)h * h)), iy = (int)((t / h) % h), iz = (int)(t % h);
        psi[(int64_t)k * M + cell_id(nc, 2 * ix + px, 2 * iy + py, 2 * iz + pz)] = stage[e];
    }
}

void launch_upward(fmmkmc_ctx *c)
{
    for (int l = c->L - 1; l >= 1; --l) {
        const int ncp = 1 << (l - 1);
        const int64_t Mp = (int64_t)ncp * ncp * ncp;
        launch(c, "m2m", k_m2m, dim3((unsigned)m2m_blocks(c->nt, ncp)), dim3(256), c->nt, ncp, c->m2m[l],
               c->phi_lv[l + 1], c->phi_lv[l]);
    }
}

void launch_downward(fmmkmc_ctx *c)
{
    const int start = c->bc == FMMKMC_PERIODIC ? 2 : 3;
    for (int l = start; l <= c->L; ++l) {
        const int nc = 1 << (l - 1);
        const int64_t Mh = (int64_t)(nc / 2) * (nc / 2) * (nc / 2);
        const double *sin_ = c->scale + (int64_t)(2 * l) * c->nt, *sout = c->scale + (int64_t)(2 * l + 1) * c->nt;
        // per-level expansions keep each level's own interaction-list terms (no L2L from the parent)
        const bool from_parent = l > start && !c->per_level;
        const double *par = from_parent ? c->psi_lv[l - 1] : nullptr;
        const int wp = from_parent ? 1 : 0, per = c->bc == FMMKMC_PERIODIC ? 1 : 0;
        if (c->nt <= 196 && Mh <= 2048) {  // small levels: 8 cells per block, for more blocks
            constexpr int C = 8;
            launch_shm(c, "m2l", k_m2l<C, 1>, dim3((unsigned)((Mh + C - 1) / C), 8), dim3(256),
                       sizeof(double) * c->nt * C, c->nt, nc, per, wp, c->m2l, c->m2l_index, sin_, sout,
                       c->l2l[l], c->phi_lv[l], par, c->psi_lv[l]);
        } else if (c->nt <= 196) {  // p <= 13: 32 cells per block, <= 50 KB of LDS
            constexpr int C = 32;
            launch_shm(c, "m2l", k_m2l<C, 1>, dim3((unsigned)((Mh + C - 1) / C), 8), dim3(256),
                       sizeof(double) * c->nt * C, c->nt, nc, per, wp, c->m2l, c->m2l_index, sin_, sout,
                       c->l2l[l], c->phi_lv[l], par, c->psi_lv[l]);
        } else {
            constexpr int C = 16;
            if (c->nt <= 256)
                launch_shm(c, "m2l", k_m2l<C, 1>, dim3((unsigned)((Mh + C - 1) / C), 8), dim3(256),
                           sizeof(double) * c->nt * C, c->nt, nc, per, wp, c->m2l, c->m2l_index, sin_, sout,
                           c->l2l[l], c->phi_lv[l], par, c->psi_lv[l]);
            else
                launch_shm(c, "m2l", k_m2l<C, 2>, dim3((unsigned)((Mh + C - 1) / C), 8), dim3(256),
                           sizeof(double) * c->nt * C, c->nt, nc, per, wp, c->m2l, c->m2l_index, sin_, sout,
                           c->l2l[l], c->phi_lv[l], par, c->psi_lv[l]);
        }
    }
}

// ---- far field -----------------------------------------------------------

// H = R K and the nonzero Chebyshev coefficients C = (G R) K.  Rows are split
// over 16 lanes each (partial sums reduced in LDS); both operators are stored
// column-major ([n][row]).
__device__ __forceinline__ void far_refresh_body(int64_t blk, int nt, int ncz, const double *__restrict__ R,
                                                 const double *__restrict__ GR, const int32_t *__restrict__ cz,
                                                 const double *__restrict__ K, double *__restrict__ H,
                                                 double *__restrict__ C)
{
    __shared__ double part[16][17];
    const int lr = threadIdx.x & 15, ls = threadIdx.x >> 4;
    const int row = (int)blk * 16 + lr;
    double acc = 0.0;
    if (row < nt + ncz) {
        const bool isH = row < nt;
        const int r = isH ? row : row - nt;
        const int ld = isH ? nt : ncz;
        const double *A = isH ? R : GR;
        for (int n = ls; n < nt; n += 16) acc += A[(int64_t)n * ld + r] * K[n];
    }
    part[ls][lr] = acc;
    __syncthreads();
    if (ls == 0 && row < nt + ncz) {
        double s = 0.0;
        for (int t = 0; t < 16; ++t) s += part[t][lr];
        if (row < nt)
            H[row] = s;
        else
            C[cz[row - nt]] = s;
    }
}

__global__ __launch_bounds__(256) void k_far_refresh(int nt, int ncz, const double *__restrict__ R,
                                                     const double *__restrict__ GR, const int32_t *__restrict__ cz,
                                                     const double *__restrict__ K, double *__restrict__ H,
                                                     double *__restrict__ C)
{
    far_refresh_body(blockIdx.x, nt, ncz, R, GR, cz, K, H, C);
}

// Chebyshev columns in two passes:
//   A[i][b][c]  = sum_{a <= p-b-c} C[a][b][c] T_a(xi_i)
//   Bz[i][j][c] = sum_{b <= p-c}   A[i][b][c] T_b(xi_j)
__device__ __forceinline__ void cheb_a_body(int64_t blk, int p, int n, const double *__restrict__ C,
                                            const double *__restrict__ Tax, double *__restrict__ A)
{
    const int q = p + 1;
    const int64_t t = blk * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * q * q) return;
    const int cc = (int)(t % q), b = (int)((t / q) % q), i = (int)(t / (q * q));
    double acc = 0.0;
    for (int a = 0; a + b + cc <= p; ++a) acc += C[(a * q + b) * q + cc] * Tax[i * q + a];
    A[t] = acc;
}

__global__ __launch_bounds__(256) void k_cheb_a(int p, int n, const double *__restrict__ C,
                                                const double *__restrict__ Tax, double *__restrict__ A)
{
    cheb_a_body(blockIdx.x, p, n, C, Tax, A);
}

__device__ __forceinline__ void cheb_b_body(int64_t blk, int p, int n, const double *__restrict__ A,
                                            const double *__restrict__ Tax, double *__restrict__ Bz)
{
    const int q = p + 1;
    const int64_t t = blk * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n * q) return;
    const int cc = (int)(t % q);
    const int64_t ij = t / q;
    const int i = (int)(ij / n), j = (int)(ij % n);
    double acc = 0.0;
    for (int b = 0; b + cc <= p; ++b) acc += A[((int64_t)i * q + b) * q + cc] * Tax[j * q + b];
    Bz[t] = acc;
}

__global__ __launch_bounds__(256) void k_cheb_b(int p, int n, const double *__restrict__ A,
                                                const double *__restrict__ Tax, double *__restrict__ Bz)
{
    cheb_b_body(blockIdx.x, p, n, A, Tax, Bz);
}

void launch_far_refresh(fmmkmc_ctx *c, hipStream_t st)
{
    if (!st) st = c->stream;
    const int q = c->p + 1, rows = c->nt + c->far.ncz;
    launch_on(c, st, "far_refresh", k_far_refresh, dim3((rows + 15) / 16), dim3(256), 0, c->nt, c->far.ncz,
              c->far.R, c->far.GR, c->far.cz, c->far.K, c->far.H, c->far.C);
    if (c->lat_n > 0) {
        const int64_t ta = (int64_t)c->lat_n * q * q, tb = (int64_t)c->lat_n * c->lat_n * q;
        launch_on(c, st, "cheb_a", k_cheb_a, dim3((unsigned)((ta + 255) / 256)), dim3(256), 0, c->p, c->lat_n,
                  c->far.C, c->far.Tax, c->far.A);
        launch_on(c, st, "cheb_b", k_cheb_b, dim3((unsigned)((tb + 255) / 256)), dim3(256), 0, c->p, c->lat_n,
                  c->far.A, c->far.Tax, c->far.Bz);
    }
}

// ---- FP32 shadow of the fine-level local expansions ------------------------

__global__ void k_to_f32(int64_t count, const double *__restrict__ in, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = (float)in[t];
}

void launch_shadow(fmmkmc_ctx *c)
{
    const int64_t tot = (int64_t)c->nt * c->M;
    launch(c, "shadow_f32", k_to_f32, dim3((unsigned)((tot + 255) / 256)), dim3(256), tot, c->psi_lv[c->L],
           c->psi32);
}


// ---- batched replicas: far-field refresh of the replicas that moved -----------

__global__ __launch_bounds__(256) void k_b_far_refresh(const RepDev *__restrict__ reps, int R,
                                                       const int64_t *__restrict__ base,
                                                       const MoveDev *__restrict__ moves)
{
    const int r = find_rep(base, R, blockIdx.x);
    if (!moves[r].valid) return;
    const RepDev &d = reps[r];
    far_refresh_body(blockIdx.x - base[r], d.nt, d.ncz, d.R, d.GR, d.cz, d.Kf, d.H, d.C);
}

__global__ __launch_bounds__(256) void k_b_cheb_a(const RepDev *__restrict__ reps, int R,
                                                  const int64_t *__restrict__ base, const MoveDev *__restrict__ moves)
{
    const int r = find_rep(base, R, blockIdx.x);
    if (!moves[r].valid) return;
    const RepDev &d = reps[r];
    cheb_a_body(blockIdx.x - base[r], d.p, d.g.n, d.C, d.Tax, d.A);
}

__global__ __launch_bounds__(256) void k_b_cheb_b(const RepDev *__restrict__ reps, int R,
                                                  const int64_t *__restrict__ base, const MoveDev *__restrict__ moves)
{
    const int r = find_rep(base, R, blockIdx.x);
    if (!moves[r].valid) return;
    const RepDev &d = reps[r];
    cheb_b_body(blockIdx.x - base[r], d.p, d.g.n, d.A, d.Tax, d.Bz);
}

void launch_b_far(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base_far,
                  int64_t blocks_far, const int64_t *base_a, int64_t blocks_a, const int64_t *base_b,
                  int64_t blocks_b, const MoveDev *moves)
{
    launch_prof(pr, st, "b_far_refresh", k_b_far_refresh, dim3((unsigned)blocks_far), dim3(256), 0, reps, R,
                base_far, moves);
    launch_prof(pr, st, "b_cheb_a", k_b_cheb_a, dim3((unsigned)blocks_a), dim3(256), 0, reps, R, base_a, moves);
    launch_prof(pr, st, "b_cheb_b", k_b_cheb_b, dim3((unsigned)blocks_b), dim3(256), 0, reps, R, base_b, moves);
}

}  // namespace fmmkmc
