// Proposal kernels: the energy change of a hop r -> r' of charge q,
//   free space (Eq. (proposed_energy)):
//     dU = q phi(r') - q phi_occ(r) - q^2 / |r' - r|
//   periodic (Eq. (proposed_energy_sr) plus the far field of Sec. 3.1):
//     dU = q phi(r') - q phi_occ(r) - q^2 sum_{nu in V_box} 1/|r' - r - a nu|
//          + q^2 (6 + 8/sqrt3 + 12/sqrt2)/a + dU_far,
// where phi(x) = Psi_{L,cell(x)}(x) + sum over the 27 (wrapped) neighbour cells
// of q_j/|x - r_j| is the potential of all charges (phi_occ leaves out the
// moving charge itself), and
//     dU_far = q (phi_inf(r') - phi_inf(r)) + 1/2 q (dphi(r') - dphi(r)),
// phi_inf the local expansion H of the copies in V_inf and dphi the change of
// that expansion when the charge moves (H -> H + R dK), i.e. the paper's
// U_inf(r') - U_inf(r) with U_inf = 1/2 E.H.
//
// On a lattice phi is evaluated once per site (every hop to a site shares it)
// and the per-slot kernel only gathers; the hop-dependent but
// charge-configuration-independent terms (self terms and the quadratic far-field
// term) are tabulated per charge and hop in F.
#include <string>

#include "batch.hpp"
#include "ewald.hpp"
#include "kernels.hpp"

namespace fmmkmc {

// ---- per-level expansions -------------------------------------------------

// The levels above the fine one (per-level mode): sum over l = lstart .. L-1 of
// Psi_l of the level-l cell holding the point, about that cell's centre.  The
// cells are the fine cell's ancestors (fine coordinates shifted right), so the
// assignment at cell faces is the fine level's.
template <int P, class PP>
__device__ inline double coarse_part(const Geo &g, PP psi_lv, double px, double py, double pz, int fx, int fy,
                                     int fz)
{
    double s = 0.0;
    for (int l = g.lstart; l < g.L; ++l) {
        const int side = 1 << (l - 1), sh = g.L - l;
        const double w = g.a / side;
        const int cx = fx >> sh, cy = fy >> sh, cz = fz >> sh;
        const int64_t Ml = (int64_t)side * side * side;
        s += l2p<P, double>(psi_lv[l] + cell_id(side, cx, cy, cz), Ml, px - (cx + 0.5) * w, py - (cy + 0.5) * w,
                            pz - (cz + 0.5) * w);
    }
    return s;
}

// ---- generic points ------------------------------------------------------

// potential at arbitrary points: local expansion + near field (+ far field);
// points are xyz[3j..3j+2] or, with pidx, the current positions of charges.
template <int P, bool MIXED>
__global__ __launch_bounds__(256) void k_point_phi(Geo g, int64_t M, int64_t m, const double *__restrict__ xyz,
                                                   const int64_t *__restrict__ pidx,
                                                   const int64_t *__restrict__ exclude,
                                                   const double *__restrict__ psi, const float *__restrict__ psi32,
                                                   const double *__restrict__ H, int with_far,
                                                   const double *__restrict__ x, const double *__restrict__ y,
                                                   const double *__restrict__ z, const double *__restrict__ q,
                                                   const int32_t *__restrict__ cnt,
                                                   const int32_t *__restrict__ slots, double *__restrict__ out,
                                                   double *const *__restrict__ psi_lv)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    double px, py, pz;
    if (pidx) {
        const int64_t i = pidx[t];
        px = x[i];
        py = y[i];
        pz = z[i];
    } else {
        px = xyz[3 * t];
        py = xyz[3 * t + 1];
        pz = xyz[3 * t + 2];
    }
    const int64_t ex = exclude ? exclude[t] : -1;
    const int cx = fine_coord(px, g.w, g.nc), cy = fine_coord(py, g.w, g.nc), cz = fine_coord(pz, g.w, g.nc);
    const int64_t cell = cell_id(g.nc, cx, cy, cz);
    const double ux = px - (cx + 0.5) * g.w, uy = py - (cy + 0.5) * g.w, uz = pz - (cz + 0.5) * g.w;
    double phi;
    if (MIXED) {
        phi = psi[cell] + (double)l2p<P, float, true>(psi32 + cell, M, (float)ux, (float)uy, (float)uz);
    } else {
        phi = l2p<P, double>(psi + cell, M, ux, uy, uz);
    }
    if (g.per_level) phi += coarse_part<P>(g, psi_lv, px, py, pz, cx, cy, cz);
    // near field over the 27 neighbour cells
    double nearv = 0.0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int ax = cx + dx, ay = cy + dy, az = cz + dz;
                double shx = 0, shy = 0, shz = 0;
                if (ax < 0 || ax >= g.nc || ay < 0 || ay >= g.nc || az < 0 || az >= g.nc) {
                    if (!g.periodic) continue;
                    shx = g.a * floordiv(ax, g.nc);
                    shy = g.a * floordiv(ay, g.nc);
                    shz = g.a * floordiv(az, g.nc);
                    ax = posmod(ax, g.nc);
                    ay = posmod(ay, g.nc);
                    az = posmod(az, g.nc);
                }
                const int64_t nb = cell_id(g.nc, ax, ay, az);
                const bool unshifted = (shx == 0 && shy == 0 && shz == 0);
                const int cn = cnt[nb];
                // mixed: each cell's charges summed in FP32, the cells in FP64
                float cellf = 0.0f;
                for (int s = 0; s < cn; ++s) {
                    const int j = slots[nb * g.cap + s];
                    if (j == ex && unshifted) continue;
                    const double ex_ = px - (x[j] + shx), ey_ = py - (y[j] + shy), ez_ = pz - (z[j] + shz);
                    if (MIXED) {
                        const float fx = (float)ex_, fy = (float)ey_, fz = (float)ez_;
                        cellf += (float)q[j] * __frsqrt_rn(fx * fx + fy * fy + fz * fz);
                    } else {
                        nearv += q[j] / sqrt(ex_ * ex_ + ey_ * ey_ + ez_ * ez_);
                    }
                }
                if (MIXED) nearv += (double)cellf;
            }
    phi += nearv;
    if (with_far) {
        const double hx = px - 0.5 * g.a, hy = py - 0.5 * g.a, hz = pz - 0.5 * g.a;
        phi += l2p<P, double>(H, 1, hx, hy, hz);
    }
    out[t] = phi;
}

void launch_point_phi(fmmkmc_ctx *c, const Geo &g, int64_t m, const double *xyz, const int64_t *pidx,
                      const int64_t *exclude, int with_far, double *out, const char *name, bool fp64)
{
    if (m <= 0) return;
    dim3 grid((unsigned)((m + 255) / 256));
    if (c->prec == FMMKMC_MIXED && !fp64) {
        FMMKMC_DISPATCH_P(c->p, launch(c, name, k_point_phi<P_, true>, grid, dim3(256), g, c->M, m, xyz, pidx,
                                       exclude, c->psi_lv[c->L], c->psi32, c->far.H, with_far, c->x, c->y, c->z,
                                       c->q, c->cell_cnt, c->cell_slots, out, (double *const *)c->d_psi_ptrs));
    } else {
        FMMKMC_DISPATCH_P(c->p, launch(c, name, k_point_phi<P_, false>, grid, dim3(256), g, c->M, m, xyz, pidx,
                                       exclude, c->psi_lv[c->L], c->psi32, c->far.H, with_far, c->x, c->y, c->z,
                                       c->q, c->cell_cnt, c->cell_slots, out, (double *const *)c->d_psi_ptrs));
    }
}

// ---- lattice sites, any cell geometry --------------------------------------

// far-field potential at lattice site (i, j, k) from the Chebyshev columns
template <int P, typename PD = const double *>
__device__ inline double far_site(int n, int i, int j, int k, PD Bz, PD Tax)
{
    const auto b = Bz + ((int64_t)i * n + j) * (P + 1);
    const auto t = Tax + (int64_t)k * (P + 1);
    double acc = 0.0;
#pragma unroll
    for (int cc = 0; cc <= P; ++cc) acc += b[cc] * t[cc];
    return acc;
}

// constexpr square root (Newton from above; exact enough for 1/sqrt of small integers)
__host__ __device__ constexpr double csqrt(double x)
{
    if (x <= 0) return 0.0;
    double r = x > 1 ? x : 1.0;
    for (int it = 0; it < 64; ++it) r = 0.5 * (r + x / r);
    return r;
}

// 1/sqrt(k) for the squared integer site offsets of the near field (kInvTab entries)
struct InvSqrtTab {
    double v[kInvTab];
    constexpr InvSqrtTab() : v{}
    {
        for (int i = 1; i < kInvTab; ++i) v[i] = 1.0 / csqrt((double)i);
    }
};

// One lane per lattice site, 256 consecutive sites (lattice order) per block,
// so every lane of a block has work whatever n is.  The near field of a site
// is the charge of every site in the 27 cells around its cell; per axis those
// cells are consecutive lattice planes (cell_rng), one run, or two when the box
// wraps around a periodic face, so the 27 cells form a box of sites whose
// offsets from the lane's site are integers, and 1/|d| = 1/(h sqrt(d^2)) comes
// from a table of integer d^2.  The site's own occupant (d^2 = 0) is left out,
// so occupied sites get phi_occ.  The union of the block's boxes (in unwrapped
// plane coordinates, where each lane's box is one range per axis) is staged in
// LDS with coalesced loads, in chunks of whole x-planes that fit the tile
// (usually one chunk), so the inner loop reads LDS instead of one scattered
// global load per (site, box site).  Only a block whose box has a single plane
// larger than the tile, or a lattice too coarse for the 1/sqrt table, reads
// the per-site array directly.  The FP64 tile keeps three blocks per CU.
constexpr int kGenSites = 256;   // sites (lanes) per block
constexpr int kTileQ = 8192;     // staged charges per block (mixed)
constexpr int kTileQ64 = 5632;   // staged charges per block (FP64)
constexpr int kTilePad = 16;     // zeros after a staged chunk: fixed-length rows read past a lane's box

template <bool MIXED>
constexpr int gen_tile_q()
{
    return MIXED ? kTileQ : kTileQ64;
}

// LDS of the general body: the 1/sqrt table and its zero half, the staged
// charges and their zero pad, the union box bounds and the longest row
template <bool MIXED>
constexpr int gen_smem_bytes()
{
    return (int)((2 * kInvTab + gen_tile_q<MIXED>() + kTilePad) * (MIXED ? sizeof(float) : sizeof(double))) + 32;
}

// Blocks of the general-lattice near field: one fine cell cx along x (the x-planes
// of that cell) and a chunk of kGenSites (y, z) sites of the plane; a plane of
// n^2 sites takes ceil(n^2 / kGenSites) chunks, lanes past its end idle.
// Lane t of chunk ch: the (y, z) site of the plane.
__device__ inline bool gen_yz(int ch, int n, int t, int &sj, int &sk)
{
    const int loc = ch * kGenSites + t;
    const bool active = loc < n * n;
    sj = active ? loc / n : 0;
    sk = active ? loc - (loc / n) * n : 0;
    return active;
}

// per-level mode: the coarse levels' potential at site s (site order), from
// g.ncoarse per-site arrays of ns entries added in array order
__device__ __forceinline__ double coarse_at(const Geo &g, gptr<const double> phic, int64_t ns, int64_t s)
{
    double v = 0.0;
    for (int a = 0; a < g.ncoarse; ++a) v += phic[(int64_t)a * ns + s];
    return v;
}

template <int P, bool MIXED>
__device__ __forceinline__ void site_general_boxrows(int si, int ch, Geo g, int64_t M, const double *__restrict__ psi_,
                                                  const float *__restrict__ psi32_, const double *__restrict__ Bz_,
                                                  const double *__restrict__ Tax_, const double *__restrict__ qsite_,
                                                  const float *__restrict__ qsite32_,
                                                  const int32_t *__restrict__ cell_rng_,
                                                  const int32_t *__restrict__ site_rank_,
                                                  double *__restrict__ phisite_, double *__restrict__ phi_r_,
                                                  const double *__restrict__ phic_, unsigned char *smem)
{
    using Real = typename std::conditional<MIXED, float, double>::type;
    constexpr InvSqrtTab IT{};
    const auto psi = as_global(psi_), Bz = as_global(Bz_), Tax = as_global(Tax_), qsite = as_global(qsite_);
    const auto psi32 = as_global(psi32_), qsite32 = as_global(qsite32_);
    const auto cell_rng = as_global(cell_rng_), site_rank = as_global(site_rank_);
    const auto phisite = as_global(phisite_), phi_r = as_global(phi_r_);
    // 1/sqrt table, then kInvTab zeros: the weight of a padded row entry
    constexpr int kTab = 2 * kInvTab;
    Real *sInv = (Real *)smem;                // kTab
    Real *sQ = sInv + kTab;                   // gen_tile_q<MIXED>() + kTilePad
    int *sLo = (int *)(sQ + gen_tile_q<MIXED>() + kTilePad), *sHi = sLo + 3, *sNz = sHi + 3;
    const int n = g.n, nc = g.nc;
    const int t = threadIdx.x;
    int sj, sk;
    const bool active = gen_yz(ch, n, t, sj, sk);  // lane 0 always is
    const int64_t s = ((int64_t)si * n + sj) * n + sk;
    for (int e = t; e < kTab; e += blockDim.x) sInv[e] = e < kInvTab ? (Real)IT.v[e] : Real(0);
    if (t < 3) {
        sLo[t] = 0x7fffffff;
        sHi[t] = -0x7fffffff;
    }
    if (t == 0) *sNz = 0;
    const gptr<const Real> Qs = MIXED ? (gptr<const Real>)qsite32 : (gptr<const Real>)qsite;
    // per axis, the planes of cells c-1, c, c+1 are at most two runs of
    // consecutive indices (two when the block wraps around a periodic face);
    // run r of an axis: planes [lo_r, hi_r] shifted by sh_r planes (empty if hi_r < lo_r)
    struct Runs {
        int lo0, hi0, sh0, lo1, hi1, sh1;
    };
    auto runs = [&](int c) {
        Runs r;
        const int a0 = c - 1 < 0 ? 0 : c - 1, a1 = c + 1 >= nc ? nc - 1 : c + 1;
        r.lo0 = cell_rng[2 * a0];
        r.hi0 = cell_rng[2 * a1 + 1];
        r.sh0 = 0;
        r.lo1 = 0;
        r.hi1 = -1;
        r.sh1 = 0;
        if (g.periodic && c - 1 < 0) {
            r.lo1 = cell_rng[2 * (nc - 1)];
            r.hi1 = cell_rng[2 * (nc - 1) + 1];
            r.sh1 = -n;
        } else if (g.periodic && c + 1 >= nc) {
            r.lo1 = cell_rng[0];
            r.hi1 = cell_rng[1];
            r.sh1 = n;
        }
        return r;
    };
    const double px = (si + 0.5) * g.h, py = (sj + 0.5) * g.h, pz = (sk + 0.5) * g.h;
    const int cx = fine_coord(px, g.w, nc), cy = fine_coord(py, g.w, nc), cz = fine_coord(pz, g.w, nc);
    Runs rx{}, ry{}, rz{};
    if (active) {
        rx = runs(cx);
        ry = runs(cy);
        rz = runs(cz);
    }
    // The lane's box in unwrapped plane coordinates: the second run of an axis
    // (the wrapped cell) adjoins the first, so the box is [blo, bhi] per axis.
    int blo[3] = {0, 0, 0}, bhi[3] = {-1, -1, -1};
    {
        const Runs *ra[3] = {&rx, &ry, &rz};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            const Runs &r = *ra[ax];
            blo[ax] = r.hi1 >= r.lo1 ? min(r.lo0 + r.sh0, r.lo1 + r.sh1) : r.lo0 + r.sh0;
            bhi[ax] = r.hi1 >= r.lo1 ? max(r.hi0 + r.sh0, r.hi1 + r.sh1) : r.hi0 + r.sh0;
        }
    }
    __syncthreads();
    if (gen_tile_q<MIXED>() > 0) {
        // union of the lanes' boxes: a butterfly over each wave (lane-varying
        // values into an LDS atomic would be serialised lane by lane), then one
        // atomic per wave
        int v[7];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            v[ax] = active ? blo[ax] : 0x7fffffff;
            v[3 + ax] = active ? bhi[ax] : -0x7fffffff;
        }
        v[6] = active ? bhi[2] - blo[2] + 1 : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int e = 0; e < 3; ++e) v[e] = min(v[e], __shfl_xor(v[e], o, 64));
#pragma unroll
            for (int e = 3; e < 7; ++e) v[e] = max(v[e], __shfl_xor(v[e], o, 64));
        }
        if ((t & 63) == 0) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                atomicMin(&sLo[ax], v[ax]);
                atomicMax(&sHi[ax], v[3 + ax]);
            }
            atomicMax(sNz, v[6]);
        }
    }
    __syncthreads();
    const int lox = sLo[0], loy = sLo[1], loz = sLo[2];
    const int Lx = sHi[0] - lox + 1, Ly = sHi[1] - loy + 1, Lz = sHi[2] - loz + 1;
    // Uniform over the block.  The union box is staged in chunks of whole
    // x-planes (usually one chunk), so every block with one plane of the box
    // within the tile takes the staged path; the staged loops read the 1/sqrt
    // table unguarded.
    const bool tiled = gen_tile_q<MIXED>() > 0 && g.tab_ok && Lx > 0 && Ly > 0 && Lz > 0 &&
                       (int64_t)Ly * Lz <= gen_tile_q<MIXED>();
    // The near field is summed per row in the working precision and the row
    // sums in FP64, so FP32 rounding does not grow with the box (mixed).
    // rowof(i, j, shx, shy, shz): the charges of plane row (i, j), indexed by z
    auto near_sum = [&](auto rowof) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int ilo = a ? rx.lo1 : rx.lo0, ihi = a ? rx.hi1 : rx.hi0, shx = a ? rx.sh1 : rx.sh0;
            for (int i = ilo; i <= ihi; ++i) {
                const int di = si - (i + shx);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int jlo = b ? ry.lo1 : ry.lo0, jhi = b ? ry.hi1 : ry.hi0, shy = b ? ry.sh1 : ry.sh0;
                    for (int j = jlo; j <= jhi; ++j) {
                        const int dj = sj - (j + shy);
                        const int dij = di * di + dj * dj;
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const int klo = e ? rz.lo1 : rz.lo0, khi = e ? rz.hi1 : rz.hi0;
                            const int shz = e ? rz.sh1 : rz.sh0;
                            const int off = sk - shz;
                            const auto row = rowof(i, j, shx, shy, shz);
                            Real racc = Real(0);
                            // 1/sqrt(0) is stored as 0: the site's own occupant drops out
                            if (g.tab_ok) {
                                // d2 = dij + (off - k)^2, stepped without multiplies
                                int d2 = dij + (off - klo) * (off - klo), st = 2 * (off - klo) - 1;
#pragma unroll 4
                                for (int k = klo; k <= khi; ++k) {
                                    racc += row[k] * sInv[d2];
                                    d2 -= st;
                                    st -= 2;
                                }
                            } else {
                                for (int k = klo; k <= khi; ++k) {
                                    const int dk = off - k;
                                    const int d2 = dij + dk * dk;
                                    const Real inv = d2 < kInvTab ? sInv[d2 < kInvTab ? d2 : 0]
                                                                  : Real(1) / sqrt((Real)d2);
                                    racc += row[k] * inv;
                                }
                            }
                            acc += (double)racc;
                        }
                    }
                }
            }
        }
        return acc;
    };
    double nearv = 0.0;
    if (tiled) {
        const int cpl = gen_tile_q<MIXED>() / (Ly * Lz);  // x-planes per chunk
        // plane coordinate u (unwrapped) -> lattice index, or -1 outside a free-space box
        auto wrap = [&](int u) { return g.periodic ? (u < 0 ? u + n : (u >= n ? u - n : u)) : (u >= 0 && u < n ? u : -1); };
        // planes x0 .. x0 + nxp - 1 of the union box into sQ, then kTilePad zeros
        auto stage = [&](int x0, int nxp) {
            const int tot = nxp * Ly * Lz;
            if (Lz <= (int)blockDim.x) {
                // each thread keeps one z of the box and walks the (x, y) rows
                // rpp at a time: no integer division per element
                const int rpp = blockDim.x / Lz, zt = t % Lz;
                int r = t / Lz;
                if (r < rpp) {
                    const int uz = wrap(loz + zt);
                    int ix = r / Ly, iy = r - (r / Ly) * Ly;
                    for (; r < nxp * Ly; r += rpp) {
                        const int ux = wrap(x0 + ix), uy = wrap(loy + iy);
                        const bool in = ux >= 0 && uy >= 0 && uz >= 0;
                        sQ[r * Lz + zt] = in ? Qs[((int64_t)ux * n + uy) * n + uz] : Real(0);
                        iy += rpp;
                        while (iy >= Ly) {
                            iy -= Ly;
                            ++ix;
                        }
                    }
                }
            } else {
                for (int e = t; e < tot; e += blockDim.x) {
                    const int ix = e / (Ly * Lz), iy = (e / Lz) % Ly, iz = e % Lz;
                    const int ux = wrap(x0 + ix), uy = wrap(loy + iy), uz = wrap(loz + iz);
                    const bool in = ux >= 0 && uy >= 0 && uz >= 0;
                    sQ[e] = in ? Qs[((int64_t)ux * n + uy) * n + uz] : Real(0);
                }
            }
            if (t < kTilePad) sQ[tot + t] = Real(0);
        };
        // The lane's rows with x in [xa, xb], p0 = the staged row (xa, blo_y)
        // at z = blo_z.  Squared x and y offsets are stepped without
        // multiplies (d^2 falls by 2d - 1 when d falls by 1).  Fixed-length
        // rows: NZ >= every lane's nz, unrolled with no remainder; entry z has
        // table index dxy^2 + off[z], off[z] = (dz0 - z)^2 for z < nz and
        // kInvTab (a zero weight) past the lane's box.
        const int nz = bhi[2] - blo[2] + 1, dz0 = sk - blo[2], dy0 = sj - blo[1];
        auto rows = [&](auto nzc, int xa, int xb, const Real *p0) {
            constexpr int NZ = decltype(nzc)::value;
            int off[NZ];
#pragma unroll
            for (int z = 0; z < NZ; ++z) off[z] = z < nz ? (dz0 - z) * (dz0 - z) : kInvTab;
            double acc = 0.0;
            const int dx0 = si - xa;
            int dx2 = dx0 * dx0, stx = 2 * dx0 - 1;
            for (int x = xa; x <= xb; ++x, p0 += Ly * Lz) {
                const Real *row = p0;
                int b = dx2 + dy0 * dy0, sty = 2 * dy0 - 1;
                for (int y = blo[1]; y <= bhi[1]; ++y, row += Lz) {
                    Real racc = Real(0);
#pragma unroll
                    for (int z = 0; z < NZ; ++z) racc += row[z] * sInv[b + off[z]];
                    acc += (double)racc;
                    b -= sty;
                    sty -= 2;
                }
                dx2 -= stx;
                stx -= 2;
            }
            return acc;
        };
        // rows of the lane's own length, d^2 stepped along z as well
        auto rows_var = [&](int xa, int xb, const Real *p0) {
            double acc = 0.0;
            const int dx0 = si - xa, stz0 = 2 * dz0 - 1;
            int dx2 = dx0 * dx0 + dz0 * dz0, stx = 2 * dx0 - 1;
            for (int x = xa; x <= xb; ++x, p0 += Ly * Lz) {
                const Real *row = p0;
                int d2y = dx2 + dy0 * dy0, sty = 2 * dy0 - 1;
                for (int y = blo[1]; y <= bhi[1]; ++y, row += Lz) {
                    int d2 = d2y, st = stz0;
                    Real racc = Real(0);
#pragma unroll 4
                    for (int z = 0; z < nz; ++z) {
                        racc += row[z] * sInv[d2];
                        d2 -= st;
                        st -= 2;
                    }
                    acc += (double)racc;
                    d2y -= sty;
                    sty -= 2;
                }
                dx2 -= stx;
                stx -= 2;
            }
            return acc;
        };
        for (int x0 = lox; x0 < lox + Lx; x0 += cpl) {
            const int nxp = min(cpl, lox + Lx - x0);
            __syncthreads();  // the previous chunk has been read
            stage(x0, nxp);
            __syncthreads();
            const int xa = max(blo[0], x0), xb = min(bhi[0], x0 + nxp - 1);
            if (active && xa <= xb) {
                const Real *p0 = sQ + ((xa - x0) * Ly + (blo[1] - loy)) * Lz + (blo[2] - loz);
                // row length: the block's longest (uniform), so that padding is
                // only the difference between its lanes
                using std::integral_constant;
                switch (*sNz) {
                case 1: case 2: case 3: case 4: nearv += rows(integral_constant<int, 4>{}, xa, xb, p0); break;
                case 5: nearv += rows(integral_constant<int, 5>{}, xa, xb, p0); break;
                case 6: nearv += rows(integral_constant<int, 6>{}, xa, xb, p0); break;
                case 7: nearv += rows(integral_constant<int, 7>{}, xa, xb, p0); break;
                case 8: nearv += rows(integral_constant<int, 8>{}, xa, xb, p0); break;
                case 9: nearv += rows(integral_constant<int, 9>{}, xa, xb, p0); break;
                case 10: nearv += rows(integral_constant<int, 10>{}, xa, xb, p0); break;
                case 11: nearv += rows(integral_constant<int, 11>{}, xa, xb, p0); break;
                case 12: nearv += rows(integral_constant<int, 12>{}, xa, xb, p0); break;
                default: nearv += rows_var(xa, xb, p0); break;
                }
            }
        }
    } else if (active) {
        // the per-site array (wrapped z)
        nearv = near_sum([&](int i, int j, int, int, int) { return Qs + ((int64_t)i * n + j) * n; });
    }
    if (!active) return;
    // phisite holds the local expansion, far-field and coarse-level part (site_lf_body)
    const double phi = phisite[s] + nearv / g.h;
    const int32_t rk = site_rank[s];
    if (rk >= 0) phi_r[rk] = phi;
    phisite[s] = rk >= 0 ? __builtin_nan("") : phi;
}

// ---- general lattice, block-uniform x-window -----------------------------
// A block holds the G x-planes of one fine cell cx and a chunk of (y, z)
// sites, so its lanes share the x-planes of the cells cx-1 .. cx+1: a window
// of NX consecutive planes (unwrapped), the same for every lane.  The union
// over the lanes of their (y, z) boxes is staged once as columns of NX
// charges, [y][z][x] with x fastest, beside a table of 1/sqrt(r + dx^2) for
// every r = dy^2 + dz^2 up to the block's largest and every x offset dx
// between the window and the G planes.  Each lane computes the G sites of its
// (y, z) position in the cell's planes: they have one box, so every column of
// NX charges is read once and the G sites take the same table row shifted by
// one entry per plane; that divides the LDS words per (site, box site) by
// about G.  A table row of zeros (r = RZ) stands for the columns of the
// block's longest box that lie outside a lane's shorter box, and 1/sqrt(0) is
// stored as 0, which leaves a site's own occupant out.  Charges are staged in
// FP32: mixed precision rounds them so, and the FP64 path takes this body
// only when every charge is exactly an FP32 number.
constexpr int kG2Tile = 10240;  // staged charges (FP32)
constexpr int kG2Tab = 1536;    // table entries (working precision)
constexpr int kG2MaxNX = 12;
constexpr int kG2MaxG = 4;

template <bool MIXED>
constexpr int g2_smem_bytes()
{
    return kG2Tile * 4 + kG2Tab * (MIXED ? 4 : 8) + 4 * 8 * 4;
}

template <bool MIXED>
constexpr int general_smem_bytes()
{
    return g2_smem_bytes<MIXED>() > gen_smem_bytes<MIXED>() ? g2_smem_bytes<MIXED>() : gen_smem_bytes<MIXED>();
}

// near-field sums of one lane's G sites: NY x NZ columns (the block's longest
// box), of which ny x nz are the lane's own; col0 its first column, (dy0,
// dz0) the offset of that column from the sites.  Table rows hold TW = NX +
// G - 1 entries: entry e is dx = e - (G - 1) + (window start - first plane),
// so plane g reads entries ix + G - 1 - g.
template <int NX, int G, typename Real>
__device__ __forceinline__ void g2_near(const float *__restrict__ tile, const Real *__restrict__ tab, int Lz,
                                        int NY, int NZ, int RZ, int col0, int ny, int nz, int dy0, int dz0,
                                        double (&acc)[G])
{
    constexpr int TW = NX + G - 1;
#pragma unroll
    for (int gi = 0; gi < G; ++gi) acc[gi] = 0.0;
    for (int yy = 0; yy < NY; ++yy) {
        const int dy = dy0 + yy;
        const int oy = yy < ny ? dy * dy : RZ;
        // a row past the lane's box weighs nothing; it reads the lane's first
        // row so that every read stays inside the staged columns
        const float *col = tile + (col0 + (yy < ny ? yy : 0) * Lz) * NX;
        int dz2 = dz0 * dz0, st = 2 * dz0 + 1;  // (d + 1)^2 = d^2 + 2d + 1
        for (int zz = 0; zz < NZ; ++zz) {
            int r = min(oy + dz2, RZ);
            r = zz < nz ? r : RZ;
            // 24-bit multiply (full rate): r * TW < 2^24
            const Real *w = (const Real *)((const char *)tab + __mul24(r, TW * (int)sizeof(Real)));
            Real c[NX], wr[TW];
#pragma unroll
            for (int ix = 0; ix < NX; ++ix) c[ix] = (Real)col[ix];
#pragma unroll
            for (int e = 0; e < TW; ++e) wr[e] = w[e];
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
                Real racc = Real(0);
#pragma unroll
                for (int ix = 0; ix < NX; ++ix) racc += c[ix] * wr[ix + G - 1 - gi];
                acc[gi] += (double)racc;
            }
            col += NX;
            dz2 += st;
            st += 2;
        }
    }
}

// The body above for block (cell cx, chunk ch); returns false (having written
// nothing) when the cell has more than kG2MaxG planes, the block's union does
// not fit the tile or the table, or the charges are not staged in FP32, and
// the caller falls back to site_general_boxrows plane by plane.
template <bool MIXED>
__device__ __forceinline__ bool site_general_g2(int cx, int ch, Geo g, const float *__restrict__ qsite32_,
                                                const int32_t *__restrict__ cell_rng_,
                                                const int32_t *__restrict__ site_rank_,
                                                double *__restrict__ phisite_, double *__restrict__ phi_r_,
                                                unsigned char *smem)
{
    using Real = typename std::conditional<MIXED, float, double>::type;
    const auto Q = as_global(qsite32_);
    const auto cell_rng = as_global(cell_rng_), site_rank = as_global(site_rank_);
    const auto phisite = as_global(phisite_), phi_r = as_global(phi_r_);
    // the table first: its rows are then addressed by small immediate offsets
    Real *tab = (Real *)smem;
    float *tile = (float *)(smem + kG2Tab * sizeof(Real));
    int *red = (int *)(smem + kG2Tab * sizeof(Real) + kG2Tile * 4);  // [4 waves][8]
    const int n = g.n, nc = g.nc, t = threadIdx.x;
    const int x0 = cell_rng[2 * cx], G = cell_rng[2 * cx + 1] - x0 + 1;  // the cell's planes
    int sj, sk;
    const bool active = gen_yz(ch, n, t, sj, sk);
    // per axis, the unwrapped planes [lo, hi] of the cells c-1 .. c+1 around
    // cell c (a periodic neighbour across a face is shifted by n)
    auto box_of = [&](int c, int &lo, int &hi) {
        const int a0 = c - 1 < 0 ? 0 : c - 1, a1 = c + 1 >= nc ? nc - 1 : c + 1;
        lo = cell_rng[2 * a0];
        hi = cell_rng[2 * a1 + 1];
        if (g.periodic && c - 1 < 0) lo = cell_rng[2 * (nc - 1)] - n;
        else if (g.periodic && c + 1 >= nc) hi = cell_rng[1] + n;
    };
    int xlo, xhi, ylo, yhi, zlo, zhi;
    const int cy = fine_coord((sj + 0.5) * g.h, g.w, nc), cz = fine_coord((sk + 0.5) * g.h, g.w, nc);
    box_of(cx, xlo, xhi);
    box_of(cy, ylo, yhi);
    box_of(cz, zlo, zhi);
    // block-wide: union of the (y, z) boxes, longest ny and nz, largest |dy|, |dz|
    int v[8];
    v[0] = active ? ylo : 0x7fffffff;
    v[1] = active ? zlo : 0x7fffffff;
    v[2] = active ? yhi : -0x7fffffff;
    v[3] = active ? zhi : -0x7fffffff;
    v[4] = active ? yhi - ylo + 1 : 0;
    v[5] = active ? zhi - zlo + 1 : 0;
    v[6] = active ? max(sj - ylo, yhi - sj) : 0;
    v[7] = active ? max(sk - zlo, zhi - sk) : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int e = 0; e < 2; ++e) v[e] = min(v[e], __shfl_xor(v[e], o, 64));
#pragma unroll
        for (int e = 2; e < 8; ++e) v[e] = max(v[e], __shfl_xor(v[e], o, 64));
    }
    if ((t & 63) == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) red[(t >> 6) * 8 + e] = v[e];
    }
    __syncthreads();
    int u[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) u[e] = red[e];
    for (int wv = 1; wv < (int)(blockDim.x >> 6); ++wv) {
#pragma unroll
        for (int e = 0; e < 2; ++e) u[e] = min(u[e], red[wv * 8 + e]);
#pragma unroll
        for (int e = 2; e < 8; ++e) u[e] = max(u[e], red[wv * 8 + e]);
    }
    const int loy = u[0], loz = u[1], Ly = u[2] - loy + 1, Lz = u[3] - loz + 1, NY = u[4], NZ = u[5];
    const int RZ = u[6] * u[6] + u[7] * u[7] + 1;
    const int NX = xhi - xlo + 1, TW = NX + G - 1;  // the same on every lane
    // the staged columns, then NZ columns of zeros: a lane's columns past its
    // shorter z-box run at most that far past the union's last column
    const bool fits = g.q32 && G <= kG2MaxG && NX <= kG2MaxNX && (Ly * Lz + NZ) * NX <= kG2Tile &&
                      (RZ + 1) * TW <= kG2Tab;
    if (!fits) {
        __syncthreads();  // every lane has read red before the fallback reuses the LDS
        return false;
    }
    // stage the columns: each thread keeps one z and walks the (x, y) rows
    auto wrap = [&](int w) {
        return g.periodic ? (w < 0 ? w + n : (w >= n ? w - n : w)) : (w >= 0 && w < n ? w : -1);
    };
    if (Lz <= (int)blockDim.x) {
        // each thread keeps one z and walks the (x, y) rows, eight loads in
        // flight before their stores
        const int rpp = blockDim.x / Lz, zt = t % Lz;
        int r = t / Lz;
        if (r < rpp) {
            const int uz = wrap(loz + zt);
            int ix = r / Ly, iy = r - (r / Ly) * Ly;
            while (r < NX * Ly) {
                float qv[8];
                int at[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool in_r = r < NX * Ly;
                    const int ux = wrap(xlo + ix), uy = wrap(loy + iy);
                    const bool ok = in_r && ux >= 0 && uy >= 0 && uz >= 0;
                    qv[u] = ok ? Q[((int64_t)ux * n + uy) * n + uz] : 0.0f;
                    at[u] = in_r ? (iy * Lz + zt) * NX + ix : -1;
                    r += rpp;
                    iy += rpp;
                    while (iy >= Ly) {
                        iy -= Ly;
                        ++ix;
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (at[u] >= 0) tile[at[u]] = qv[u];
            }
        }
    } else {
        for (int e = t; e < NX * Ly * Lz; e += blockDim.x) {
            const int ix = e / (Ly * Lz), iy = (e / Lz) % Ly, iz = e % Lz;
            const int ux = wrap(xlo + ix), uy = wrap(loy + iy), uz = wrap(loz + iz);
            float qv = 0.0f;
            if (ux >= 0 && uy >= 0 && uz >= 0) qv = Q[((int64_t)ux * n + uy) * n + uz];
            tile[(iy * Lz + iz) * NX + ix] = qv;
        }
    }
    for (int e = t; e < NZ * NX; e += blockDim.x) tile[Ly * Lz * NX + e] = 0.0f;
    // table: row r, entry e holds 1/sqrt(r + dx^2), dx = xlo - x0 - (G - 1) + e; row RZ is zeros
    for (int e = t; e < (RZ + 1) * TW; e += blockDim.x) {
        const int r = e / TW, ix = e - (e / TW) * TW;
        const int dx = xlo - x0 - (G - 1) + ix;
        const int d2 = r + dx * dx;
        tab[e] = (r >= RZ || d2 == 0) ? Real(0) : (Real)(1.0 / sqrt((double)d2));
    }
    __syncthreads();
    if (!active) return true;
    const int col0 = (ylo - loy) * Lz + (zlo - loz);
    const int ny = yhi - ylo + 1, nz = zhi - zlo + 1, dy0 = ylo - sj, dz0 = zlo - sk;
    double acc[kG2MaxG];
    switch (G * 16 + NX) {
#define FMMKMC_G2_CASE(gg, k)                                                                                    \
    case gg * 16 + k: {                                                                                          \
        double a_[gg];                                                                                           \
        g2_near<k, gg, Real>(tile, tab, Lz, NY, NZ, RZ, col0, ny, nz, dy0, dz0, a_);                             \
        for (int gi = 0; gi < gg; ++gi) acc[gi] = a_[gi];                                                        \
    } break;
#define FMMKMC_G2_ROW(gg)                                                                                        \
    FMMKMC_G2_CASE(gg, 1) FMMKMC_G2_CASE(gg, 2) FMMKMC_G2_CASE(gg, 3) FMMKMC_G2_CASE(gg, 4)                       \
    FMMKMC_G2_CASE(gg, 5) FMMKMC_G2_CASE(gg, 6) FMMKMC_G2_CASE(gg, 7) FMMKMC_G2_CASE(gg, 8)                       \
    FMMKMC_G2_CASE(gg, 9) FMMKMC_G2_CASE(gg, 10) FMMKMC_G2_CASE(gg, 11) FMMKMC_G2_CASE(gg, 12)
    FMMKMC_G2_ROW(1) FMMKMC_G2_ROW(2) FMMKMC_G2_ROW(3) FMMKMC_G2_ROW(4)
#undef FMMKMC_G2_ROW
#undef FMMKMC_G2_CASE
    default:
        for (int gi = 0; gi < kG2MaxG; ++gi) acc[gi] = 0.0;
        break;
    }
    for (int gi = 0; gi < G; ++gi) {
        const int64_t s = ((int64_t)(x0 + gi) * n + sj) * n + sk;
        // phisite holds the local expansion, far-field and coarse-level part (site_lf_body)
        const double phi = phisite[s] + acc[gi] / g.h;
        const int32_t rk = site_rank[s];
        if (rk >= 0) phi_r[rk] = phi;
        phisite[s] = rk >= 0 ? __builtin_nan("") : phi;
    }
    return true;
}

// General lattices, first pass: the part of a site's potential that is not
// the near field: L2P of its fine cell's local expansion, the coarser levels
// (per-level mode) and the far field.  The near-field pass adds its sum to
// this value.  Blocks as in the near-field pass: one fine cell cx along x and
// a chunk of (y, z) sites; a lane takes the cell's G planes at its (y, z), one
// fine cell, so in mixed precision it reads each coefficient once for G sites.
template <int P, typename Real, int G>
__device__ __forceinline__ void lf_planes(const Geo &g, gptr<const Real> src, int64_t M, int64_t cell, int x0,
                                          double cxw, Real uy, Real uz, double (&out)[G])
{
    Real ux[G], v[G];
#pragma unroll
    for (int q = 0; q < G; ++q) ux[q] = (Real)((x0 + q + 0.5) * g.h - cxw);
    auto L = [&](int k) { return (src + (int64_t)k * M)[(uint32_t)cell]; };
    l2p_fn_x<P, Real, G, std::is_same<Real, float>::value>(L, ux, uy, uz, v);
#pragma unroll
    for (int q = 0; q < G; ++q) out[q] = (double)v[q];
}

template <int P, bool MIXED>
__device__ __forceinline__ void site_lf_body(int64_t blk, Geo g, int64_t M, const double *__restrict__ psi_,
                                             const float *__restrict__ psi32_, const double *__restrict__ Bz_,
                                             const double *__restrict__ Tax_, const int32_t *__restrict__ cell_rng_,
                                             const double *__restrict__ phic_, double *__restrict__ phisite_)
{
    using Real = typename std::conditional<MIXED, float, double>::type;
    const int n = g.n, nc = g.nc, t = threadIdx.x;
    const int bpp = (n * n + kGenSites - 1) / kGenSites;
    const int cx = (int)(blk / bpp), ch = (int)(blk - (int64_t)cx * bpp);
    int sj, sk;
    if (!gen_yz(ch, n, t, sj, sk)) return;
    const auto cell_rng = as_global(cell_rng_);
    const int x0 = cell_rng[2 * cx], G = cell_rng[2 * cx + 1] - x0 + 1;  // the cell's planes
    const auto psi = as_global(psi_), Bz = as_global(Bz_), Tax = as_global(Tax_);
    const gptr<const Real> src = MIXED ? (gptr<const Real>)as_global(psi32_) : (gptr<const Real>)as_global(psi_);
    const double py = (sj + 0.5) * g.h, pz = (sk + 0.5) * g.h;
    const int cy = fine_coord(py, g.w, nc), cz = fine_coord(pz, g.w, nc);
    const int64_t cell = cell_id(nc, cx, cy, cz);
    const double cxw = (cx + 0.5) * g.w;
    const Real uy = (Real)(py - (cy + 0.5) * g.w), uz = (Real)(pz - (cz + 0.5) * g.w);
    const double c0 = MIXED ? psi[cell] : 0.0;  // mixed: the constant term in FP64
    auto finish = [&](int q, double l) {
        const int si = x0 + q;
        const int64_t s = ((int64_t)si * n + sj) * n + sk;
        double phi = c0 + l;
        if (phic_) phi += coarse_at(g, as_global(phic_), (int64_t)n * n * n, s);  // per-level mode: the coarser levels
        if (g.periodic) phi += far_site<P>(n, si, sj, sk, Bz, Tax);
        as_global(phisite_)[s] = phi;
    };
    auto run = [&](auto gc) {
        constexpr int GG = decltype(gc)::value;
        double o[GG];
        lf_planes<P, Real, GG>(g, src, M, cell, x0, cxw, uy, uz, o);
#pragma unroll
        for (int q = 0; q < GG; ++q) finish(q, o[q]);
    };
    using std::integral_constant;
    // FP64: one site at a time (the shared form's registers cost more occupancy than its loads save)
    switch (MIXED ? G : 0) {
    case 1: run(integral_constant<int, 1>{}); break;
    case 2: run(integral_constant<int, 2>{}); break;
    case 3: run(integral_constant<int, 3>{}); break;
    case 4: run(integral_constant<int, 4>{}); break;
    default:
        // one site at a time
        for (int q = 0; q < G; ++q) {
            double o[1];
            lf_planes<P, Real, 1>(g, src, M, cell, x0 + q, cxw, uy, uz, o);
            finish(q, o[0]);
        }
        break;
    }
}

template <int P, bool MIXED>
__global__ __launch_bounds__(256) void k_site_lf(Geo g, int64_t M, const double *__restrict__ psi,
                                                 const float *__restrict__ psi32, const double *__restrict__ Bz,
                                                 const double *__restrict__ Tax, const int32_t *__restrict__ cell_rng,
                                                 const double *__restrict__ phic, double *__restrict__ phisite)
{
    site_lf_body<P, MIXED>(blockIdx.x, g, M, psi, psi32, Bz, Tax, cell_rng, phic, phisite);
}

// a general-lattice block (fine cell cx along x, chunk ch of (y, z) sites):
// the x-window body, else the box-row body for each plane of the cell
template <int P, bool MIXED>
__device__ __forceinline__ void site_general_body(int64_t blk, Geo g, int64_t M, const double *__restrict__ psi,
                                                  const float *__restrict__ psi32, const double *__restrict__ Bz,
                                                  const double *__restrict__ Tax, const double *__restrict__ qsite,
                                                  const float *__restrict__ qsite32,
                                                  const int32_t *__restrict__ cell_rng,
                                                  const int32_t *__restrict__ site_rank, double *__restrict__ phisite,
                                                  double *__restrict__ phi_r, const double *__restrict__ phic,
                                                  unsigned char *smem)
{
    const int bpp = (g.n * g.n + kGenSites - 1) / kGenSites;
    const int cx = (int)(blk / bpp), ch = (int)(blk - (int64_t)cx * bpp);
    if (site_general_g2<MIXED>(cx, ch, g, qsite32, cell_rng, site_rank, phisite, phi_r, smem)) return;
    const int x0 = as_global(cell_rng)[2 * cx], x1 = as_global(cell_rng)[2 * cx + 1];
    for (int si = x0; si <= x1; ++si) {
        site_general_boxrows<P, MIXED>(si, ch, g, M, psi, psi32, Bz, Tax, qsite, qsite32, cell_rng, site_rank,
                                       phisite, phi_r, phic, smem);
        __syncthreads();  // the next plane restages the LDS
    }
}

// blocks of the general-lattice near field: fine cells along x times chunks of a plane
int64_t general_site_blocks(int n, int nc)
{
    return (int64_t)nc * ((n * n + kGenSites - 1) / kGenSites);
}

template <int P, bool MIXED>
__global__ __launch_bounds__(256) void k_site_phi_general(Geo g, int64_t M, const double *__restrict__ psi,
                                                          const float *__restrict__ psi32,
                                                          const double *__restrict__ Bz,
                                                          const double *__restrict__ Tax,
                                                          const double *__restrict__ qsite,
                                                          const float *__restrict__ qsite32,
                                                          const int32_t *__restrict__ cell_rng,
                                                          const int32_t *__restrict__ site_rank,
                                                          double *__restrict__ phisite, double *__restrict__ phi_r,
                                                          const double *__restrict__ phic)
{
    __shared__ __align__(16) unsigned char smem[general_smem_bytes<MIXED>()];
    site_general_body<P, MIXED>(blockIdx.x, g, M, psi, psi32, Bz, Tax, qsite, qsite32, cell_rng, site_rank,
                                phisite, phi_r, phic, smem);
}

// ---- lattice with 2 x 2 x 2 sites per fine cell ----------------------------
// One lane per fine cell, 8 sites at offsets (+-h/2, +-h/2, +-h/2) from the
// centre.  Reflections of a site offset map the L2P weights onto each other:
//   x -> -x: R_n^m -> (-1)^m conj(R_n^m),  y -> -y: R_n^m -> conj(R_n^m),
//   z -> -z: R_n^m -> (-1)^(n+m) R_n^m,
// so the 8 potentials follow from 8 sums (classes by the parities of m and
// n + m, real or imaginary part) of one weight vector, that of (h/2)(1,1,1).
// Those weights at unit spacing and the near-field 1/|d| for the offsets of
// the 27-cell block are compile-time constants; only the powers h^n and 1/h
// are applied at run time.  No tables are read.


template <int P>
struct S2Weights {
    double w[nterms(P)];  // L2P weights at (1/2, 1/2, 1/2)
    constexpr S2Weights() : w{}
    {
        const double x = 0.5, y = 0.5, z = 0.5, r2 = 0.75;
        double cm2 = 1.0, cm1 = z;
        w[0] = 1.0;
        if (P >= 1) w[slot0(1)] = z;
        for (int n = 2; n <= P; ++n) {
            const double c = ((2 * n - 1) * z * cm1 - r2 * cm2) / ((double)(n * n));
            w[slot0(n)] = c;
            cm2 = cm1;
            cm1 = c;
        }
        double dr = 1.0, di = 0.0;
        for (int m = 1; m <= P; ++m) {
            const double f = -0.5 / m;
            const double ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
            dr = ndr;
            di = ndi;
            double ar = dr, ai = di;
            w[slot_re(m, m)] = 2 * ar;
            w[slot_im(m, m)] = 2 * ai;
            if (m + 1 > P) continue;
            double br = z * ar, bi = z * ai;
            w[slot_re(m + 1, m)] = 2 * br;
            w[slot_im(m + 1, m)] = 2 * bi;
            for (int n = m + 2; n <= P; ++n) {
                const double q = 1.0 / ((double)((n + m) * (n - m)));
                const double cr = ((2 * n - 1) * z * br - r2 * ar) * q;
                const double ci = ((2 * n - 1) * z * bi - r2 * ai) * q;
                w[slot_re(n, m)] = 2 * cr;
                w[slot_im(n, m)] = 2 * ci;
                ar = br;
                ai = bi;
                br = cr;
                bi = ci;
            }
        }
    }
};

// 1 / sqrt(d2) for the squared offsets of the 27-cell block (d2 <= 27)
struct InvSqrt {
    double v[28];
    constexpr InvSqrt() : v{}
    {
        for (int i = 1; i < 28; ++i) v[i] = 1.0 / csqrt((double)i);
    }
};

// squared offset (unit spacing) between site u of a cell and site v of neighbour nb
__host__ __device__ constexpr int s2_d2(int u, int nb, int v)
{
    const int dx = 2 * (nb / 9 - 1) + (v >> 2) - (u >> 2);
    const int dy = 2 * ((nb / 3) % 3 - 1) + ((v >> 1) & 1) - ((u >> 1) & 1);
    const int dz = 2 * (nb % 3 - 1) + (v & 1) - (u & 1);
    return dx * dx + dy * dy + dz * dz;
}

// near-field terms of neighbour cell NB at the 8 sites of a cell: compile-time
// 1/|d| (unit spacing), so no lane reads a weight from memory
template <int NB, typename Real>
__device__ __forceinline__ void s2_near_cell(const Real (&qv)[8], double (&near_)[8])
{
    constexpr InvSqrt IS{};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        Real part = Real(0);
#pragma unroll
        for (int v = 0; v < 8; ++v) part += (Real)IS.v[s2_d2(u, NB, v)] * qv[v];
        near_[u] += (double)part;
    }
}

// neighbour nb (uniform over the wave): one branch to its compile-time weights
template <typename Real, int... NBs>
__device__ __forceinline__ void s2_near_switch(int nb, const Real (&qv)[8], double (&near_)[8],
                                               std::integer_sequence<int, NBs...>)
{
    (void)((nb == NBs ? (s2_near_cell<NBs, Real>(qv, near_), true) : false) || ...);
}

// The two kinds of work have different shapes: the class sums stream
// (p+1)^2 coefficients per cell from HBM, the near field walks 27 neighbour
// cells through L2, and both are bound by how many loads a CU keeps in flight.
// Every lane of a block takes part in both, one after the other: two lanes per
// cell (lane t and t + CELLS, so each SIMD holds a wave of either half), which
// first split the cell's degrees for the class sums (the low degrees, about
// half the coefficients, and the rest) and then its 27 neighbour cells for the
// near field.  Each pair adds its two partial sums through LDS, and all waves
// write the block's sites contiguously.  An earlier form gave half of the
// waves the class sums and the other half the near field; timed apart, the
// class-sum waves took twice as long as the near-field waves.  Sharing both
// phases among all waves measured the same in FP64 (114 us at 128^3, L = 7,
// p = 12) and 4 % faster in mixed precision (96 -> 92 us): the class sums
// stream Psi_L at about 3.5 TB/s either way.
template <int NW>
constexpr int s2_cells() { return 32 * NW; }  // cells per block (2 lanes per cell)

// LDS of the 2x2x2 body: the two per-site results (rows of 9: no bank conflicts)
template <bool MIXED, int NW>
constexpr int s2_smem_bytes()
{
    return 2 * s2_cells<NW>() * 9 * 8;
}

// first degree of the second half of the class sums: about half the (p+1)^2 coefficients below it
__host__ __device__ constexpr int s2_degree_split(int P)
{
    int n = 0;
    while (2 * n * n < (P + 1) * (P + 1)) ++n;
    return n;
}

// class sums S[A][B][C] over degrees N0 .. N1 - 1 of one cell: A = (n+m) & 1,
// B = m & 1, C = 0 real part / 1 imaginary part.  Each degree is summed in the
// working precision and the degrees in FP64, so in mixed precision the
// rounding does not grow with the order.
template <int P, bool MIXED, int N0, int N1, typename Real, class PS>
__device__ __forceinline__ void s2_class_sums(PS Ps, int64_t M, int64_t cell, Real h, double (&S)[2][2][2])
{
    constexpr S2Weights<P> W{};
    Real hn = Real(1);
#pragma unroll
    for (int n = 0; n < N0; ++n) hn *= h;
#pragma unroll
    for (int n = N0; n < N1; ++n) {
        Real part[2][2] = {};  // [B][C] within degree n
        Real v[2 * P + 1];
#pragma unroll
        for (int k = 0; k < 2 * n + 1; ++k) v[k] = (MIXED && n == 0) ? Real(0) : Ps[(int64_t)(n * n + k) * M + cell];
#pragma unroll
        for (int k = 0; k < 2 * n + 1; ++k) {
            const int m = (k + 1) / 2, C = (k > 0 && (k & 1) == 0) ? 1 : 0;
            part[m & 1][C] += (Real)W.w[n * n + k] * v[k];
        }
#pragma unroll
        for (int B = 0; B < 2; ++B)
#pragma unroll
            for (int C = 0; C < 2; ++C) S[(n + B) & 1][B][C] += (double)(hn * part[B][C]);
        hn *= h;
    }
}

template <int P, bool MIXED, int NW>
__device__ __forceinline__ void site_s2_body(int64_t blk, Geo g, int64_t M, const double *__restrict__ psi_,
                                             const float *__restrict__ psi32_, const double *__restrict__ qsite_,
                                             const float *__restrict__ qsite32_,
                                             const int32_t *__restrict__ site_rank_, const double *__restrict__ Bz_,
                                             const double *__restrict__ Tax_, double *__restrict__ phisite_,
                                             double *__restrict__ phi_r_, const double *__restrict__ phic_,
                                             unsigned char *smem)
{
    using Real = typename std::conditional<MIXED, float, double>::type;
    const auto psi = as_global(psi_), Bz = as_global(Bz_), Tax = as_global(Tax_), qsite = as_global(qsite_);
    const auto psi32 = as_global(psi32_), qsite32 = as_global(qsite32_);
    const auto site_rank = as_global(site_rank_);
    const auto phisite = as_global(phisite_), phi_r = as_global(phi_r_);
    // per cell and site: local-expansion part, near + far-field part; the second
    // half's partial sums pass through sNear before the final values
    constexpr int CELLS = s2_cells<NW>();
    double *sFar = (double *)smem, *sNear = sFar + CELLS * 9;
    static_assert(NW == 8, "2 lanes per cell: 8 waves of 64 for 256 cells");
    // per-level mode: this thread's sites' coarse-level sums, loaded now so that
    // their latency hides behind the work below
    constexpr int PER = CELLS * 8 / (64 * NW);
    double pcv[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int64_t e = threadIdx.x + (int64_t)t * blockDim.x;
        pcv[t] = (phic_ && blk * CELLS * 8 + e < M * 8) ? coarse_at(g, as_global(phic_), M * 8, blk * CELLS * 8 + e)
                                                        : 0.0;
    }
    const int half = (int)threadIdx.x >= CELLS ? 1 : 0;  // uniform over each wave
    const int lc = (int)threadIdx.x - half * CELLS;
    const int64_t c0 = blk * CELLS, cell = c0 + lc;
    const bool live = cell < M;
    const int nc = g.nc;
    // ---- class sums: degrees below the split on the first half, the rest on the second
    {
        constexpr int NS = s2_degree_split(P);
        const gptr<const Real> Ps = MIXED ? (gptr<const Real>)psi32 : (gptr<const Real>)psi;
        double S[2][2][2] = {};
        if (live) {
            if (half == 0)
                s2_class_sums<P, MIXED, 0, NS, Real>(Ps, M, cell, (Real)g.h, S);
            else
                s2_class_sums<P, MIXED, NS, P + 1, Real>(Ps, M, cell, (Real)g.h, S);
        }
        if (half == 1 && live) {
#pragma unroll
            for (int e = 0; e < 8; ++e) sNear[lc * 9 + e] = S[e >> 2][(e >> 1) & 1][e & 1];
        }
        __syncthreads();
        if (half == 0 && live) {
#pragma unroll
            for (int e = 0; e < 8; ++e) S[e >> 2][(e >> 1) & 1][e & 1] += sNear[lc * 9 + e];
            const double l00 = MIXED ? psi[cell] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int fx = 1 - (u >> 2), fy = 1 - ((u >> 1) & 1), fz = 1 - (u & 1);
                double far_ = 0.0;
#pragma unroll
                for (int A = 0; A < 2; ++A)
#pragma unroll
                    for (int B = 0; B < 2; ++B) {
                        const double sz = (fz && A) ? -1.0 : 1.0;
                        const double sre = sz * ((fx && B) ? -1.0 : 1.0);
                        const double sim = sz * ((fx && !B) ? -1.0 : 1.0) * (fy ? -1.0 : 1.0);
                        far_ += sre * S[A][B][0] + sim * S[A][B][1];
                    }
                sFar[lc * 9 + u] = l00 + far_;
            }
        }
        __syncthreads();  // the partials have been read before sNear takes the near-field ones
    }
    // ---- near field: neighbour cells 0 .. 12 and the far field on the first half, 13 .. 26 on the second
    {
        const gptr<const Real> Qs = MIXED ? (gptr<const Real>)qsite32 : (gptr<const Real>)qsite;
        const int cx = (int)(cell / ((int64_t)nc * nc)), cy = (int)((cell / nc) % nc), cz = (int)(cell % nc);
        // the 27 neighbour cells' 8 sites each (wrapped, or absent in free space);
        // the next cell's charges are loaded while the current one is summed
        auto cell_base = [&](int nb, bool &ok) {
            int ax = cx + nb / 9 - 1, ay = cy + (nb / 3) % 3 - 1, az = cz + nb % 3 - 1;
            ok = g.periodic || (ax >= 0 && ax < nc && ay >= 0 && ay < nc && az >= 0 && az < nc);
            ax += ax < 0 ? nc : (ax >= nc ? -nc : 0);
            ay += ay < 0 ? nc : (ay >= nc ? -nc : 0);
            az += az < 0 ? nc : (az >= nc ? -nc : 0);
            return cell_id(nc, ax, ay, az) * 8;
        };
        // a cell's 8 charges are contiguous and 64-byte aligned: vector loads.
        // The wrapped address is always inside the table, so the loads are
        // unconditional (no branch per load) and an absent cell is zeroed after.
        auto load8 = [&](int64_t base, bool ok, Real *o) {
            // builtin vector types: the HIP wrapper types cannot be copied
            // out of a global-space reference
            typedef float vf4 __attribute__((ext_vector_type(4)));
            typedef double vd2 __attribute__((ext_vector_type(2)));
            if constexpr (MIXED) {
                const gptr<const vf4> q4 = (gptr<const vf4>)(Qs + base);
                const vf4 a0 = q4[0], a1 = q4[1];
                o[0] = a0.x, o[1] = a0.y, o[2] = a0.z, o[3] = a0.w;
                o[4] = a1.x, o[5] = a1.y, o[6] = a1.z, o[7] = a1.w;
            } else {
                const gptr<const vd2> q2 = (gptr<const vd2>)(Qs + base);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const vd2 a = q2[t];
                    o[2 * t] = a.x;
                    o[2 * t + 1] = a.y;
                }
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) o[v] = ok ? o[v] : Real(0);
        };
        // each neighbour cell's 8 terms per site in the working precision, the cells in FP64
        double near_[8] = {};
        double fs[8] = {};
        if (live) {
            const int nb0 = half ? 13 : 0, nb1 = half ? 27 : 13;
            Real qn[8];
            {
                bool ok;
                const int64_t b0 = cell_base(nb0, ok);
                load8(b0, ok, qn);
            }
#pragma unroll 1
            for (int nb = nb0; nb < nb1; ++nb) {
                Real qv[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) qv[v] = qn[v];
                if (nb + 1 < nb1) {
                    bool ok;
                    const int64_t b1 = cell_base(nb + 1, ok);
                    load8(b1, ok, qn);
                }
                s2_near_switch<Real>(nb, qv, near_, std::make_integer_sequence<int, 27>{});
            }
            // far field of V_inf at the 8 sites: the 4 (i, j) rows of Bz against the two Tax rows 2cz, 2cz+1
            if (g.periodic && half == 0) {
                const int n = g.n;
                const auto t0 = Tax + (int64_t)(2 * cz) * (P + 1);
#pragma unroll
                for (int ij = 0; ij < 4; ++ij) {
                    const int i = 2 * cx + (ij >> 1), j = 2 * cy + (ij & 1);
                    const auto bz = Bz + ((int64_t)i * n + j) * (P + 1);
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int cc = 0; cc <= P; ++cc) {
                        const double bb = bz[cc];
                        a0 += bb * t0[cc];
                        a1 += bb * t0[P + 1 + cc];
                    }
                    fs[2 * ij] = a0;
                    fs[2 * ij + 1] = a1;
                }
            }
        }
        if (half == 1 && live) {
#pragma unroll
            for (int u = 0; u < 8; ++u) sNear[lc * 9 + u] = near_[u];
        }
        __syncthreads();
        if (half == 0 && live) {
            const double inv_h = 1.0 / g.h;
#pragma unroll
            for (int u = 0; u < 8; ++u) sNear[lc * 9 + u] = (near_[u] + sNear[lc * 9 + u]) * inv_h + fs[u];
        }
    }
    __syncthreads();
    const int nsite = (int)((M - c0 < CELLS ? M - c0 : CELLS) * 8);
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int e = threadIdx.x + t * blockDim.x;
        if (e >= nsite) break;
        const int l = e >> 3, u = e & 7;
        const double phi = sFar[l * 9 + u] + sNear[l * 9 + u] + pcv[t];  // + the coarser levels (per-level mode)
        const int32_t rk = site_rank[c0 * 8 + e];
        if (rk >= 0) phi_r[rk] = phi;
        phisite[c0 * 8 + e] = rk >= 0 ? __builtin_nan("") : phi;
    }
}

template <int P, bool MIXED>
__global__ __launch_bounds__(512) void k_site_phi_s2(Geo g, int64_t M, const double *__restrict__ psi,
                                                     const float *__restrict__ psi32,
                                                     const double *__restrict__ qsite,
                                                     const float *__restrict__ qsite32,
                                                     const int32_t *__restrict__ site_rank,
                                                     const double *__restrict__ Bz, const double *__restrict__ Tax,
                                                     double *__restrict__ phisite, double *__restrict__ phi_r,
                                                     const double *__restrict__ phic)
{
    __shared__ __align__(16) unsigned char smem[s2_smem_bytes<MIXED, 8>()];
    site_s2_body<P, MIXED, 8>(blockIdx.x, g, M, psi, psi32, qsite, qsite32, site_rank, Bz, Tax, phisite, phi_r,
                              phic, smem);
}

void launch_site_phi(fmmkmc_ctx *c, const Geo &g)
{
    const bool mixed = c->prec == FMMKMC_MIXED;
    if (c->s2) {
        dim3 grid((unsigned)((c->M + s2_cells<8>() - 1) / s2_cells<8>()));
        if (mixed) {
            FMMKMC_DISPATCH_P(c->p, launch(c, "site_phi_s2", k_site_phi_s2<P_, true>, grid, dim3(512), g, c->M,
                                           c->psi_lv[c->L], c->psi32, c->qsite, c->qsite32, c->site_rank, c->far.Bz,
                                           c->far.Tax, c->phisite, c->phi_r, c->phicoarse));
        } else {
            FMMKMC_DISPATCH_P(c->p, launch(c, "site_phi_s2", k_site_phi_s2<P_, false>, grid, dim3(512), g, c->M,
                                           c->psi_lv[c->L], c->psi32, c->qsite, c->qsite32, c->site_rank, c->far.Bz,
                                           c->far.Tax, c->phisite, c->phi_r, c->phicoarse));
        }
    } else {
        const dim3 glf((unsigned)general_site_blocks(c->lat_n, c->nc));
        if (mixed) {
            FMMKMC_DISPATCH_P(c->p, launch(c, "site_phi", k_site_lf<P_, true>, glf, dim3(256), g, c->M,
                                           c->psi_lv[c->L], c->psi32, c->far.Bz, c->far.Tax, c->cell_rng,
                                           c->phicoarse, c->phisite));
        } else {
            FMMKMC_DISPATCH_P(c->p, launch(c, "site_phi", k_site_lf<P_, false>, glf, dim3(256), g, c->M,
                                           c->psi_lv[c->L], c->psi32, c->far.Bz, c->far.Tax, c->cell_rng,
                                           c->phicoarse, c->phisite));
        }
        dim3 grid((unsigned)general_site_blocks(c->lat_n, c->nc));
        if (mixed) {
            FMMKMC_DISPATCH_P(c->p, launch(c, "site_phi", k_site_phi_general<P_, true>, grid, dim3(256), g, c->M,
                                           c->psi_lv[c->L], c->psi32, c->far.Bz, c->far.Tax, c->qsite, c->qsite32,
                                           c->cell_rng, c->site_rank, c->phisite, c->phi_r, c->phicoarse));
        } else {
            FMMKMC_DISPATCH_P(c->p, launch(c, "site_phi", k_site_phi_general<P_, false>, grid, dim3(256), g, c->M,
                                           c->psi_lv[c->L], c->psi32, c->far.Bz, c->far.Tax, c->qsite, c->qsite32,
                                           c->cell_rng, c->site_rank, c->phisite, c->phi_r, c->phicoarse));
        }
    }
}

// ---- per-level mode: the coarser levels at every lattice site ----------------
//
// phicoarse[s] = sum over l = lstart .. L-1 of Psi_l at site s (site order of
// the site kernels).  Any lattice: one lane per site, every coarse level.

template <int P>
__device__ inline void coarse_site_body(const Geo &g, double *const *psi_lv, int64_t s, int s2,
                                        double *__restrict__ phic)
{
    const int n = g.n;
    const int64_t ns = (int64_t)n * n * n;
    if (s >= ns) return;
    const int i = (int)(s / ((int64_t)n * n)), j = (int)((s / n) % n), k = (int)(s % n);
    const double px = (i + 0.5) * g.h, py = (j + 0.5) * g.h, pz = (k + 0.5) * g.h;
    const int fx = fine_coord(px, g.w, g.nc), fy = fine_coord(py, g.w, g.nc), fz = fine_coord(pz, g.w, g.nc);
    const double v = coarse_part<P>(g, psi_lv, px, py, pz, fx, fy, fz);
    phic[s2 ? s2_site(g.nc, i, j, k) : s] = v;
}

template <int P>
__global__ __launch_bounds__(256) void k_coarse_sites(Geo g, double *const *__restrict__ psi_lv, int s2,
                                                      double *__restrict__ phic)
{
    coarse_site_body<P>(g, psi_lv, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, s2, phic);
}

// 2 x 2 x 2 sites per fine cell: a level-l cell holds W = 2^(L-l+1) sites per
// axis, symmetric about its centre, so its sites fall into orbits of 8 under
// the reflections x, y, z -> -x, -y, -z about the centre.  Reflecting maps
// R_n^m to (-1)^m conj(R_n^m) (x), conj(R_n^m) (y) and (-1)^(n+m) R_n^m (z), so
// the 8 values of an orbit are signed sums of 8 class sums of one set of
// regular harmonics (classes: n+m parity, m parity, real or imaginary part).
// One lane per (level-l cell, orbit); the orbit's base offset is
// ((bx + 1/2) h, (by + 1/2) h, (bz + 1/2) h), bx, by, bz in [0, W/2).  A block
// covers whole cells (or a part of one cell's orbits) and first stages their
// coefficients in LDS with coalesced loads.  Every coarse level is one launch,
// each level writing its own per-site array (the site kernels add them).
// 128 lanes per block: one cell's orbits in chunks of 128, or 128 / orbits whole
// cells (their staged coefficients then take at most 16 x (p+1)^2 doubles)
constexpr int kCoarseThreads = 128;
__host__ __device__ inline int coarse_cells_per_block(int64_t orbits)
{
    return orbits >= kCoarseThreads ? 1 : (int)(kCoarseThreads / orbits);
}

// Regular harmonics carried rescaled along each column m: R_n^m = c_n Q_n with
// c_m = c_{m+1} = 1 and c_n = c_{n-2} / ((n+m)(n-m)), so the three-term step
// becomes Q_n = (g_n z) Q_{n-1} - r^2 Q_{n-2} with g_n = (2n-1) c_{n-1} / c_{n-2}
// (one multiply shared by the real and imaginary parts, then a multiply and a
// fused multiply-add each).  stage[k] folds c_n^m and the factor 2 of the
// m > 0 terms into the coefficients when they are staged.
template <int P>
struct ScaledRegular {
    double g[P + 1][P + 1];
    double stage[(P + 1) * (P + 1)];
    constexpr ScaledRegular() : g{}, stage{}
    {
        for (int m = 0; m <= P; ++m) {
            double c2 = 1.0, c1 = 1.0;  // c_{n-2}, c_{n-1}
            for (int n = m; n <= P; ++n) {
                double cn = 1.0;
                if (n >= m + 2) {
                    cn = c2 / (double)((n + m) * (n - m));
                    g[n][m] = (double)(2 * n - 1) * c1 / c2;
                }
                const double f = m > 0 ? 2.0 : 1.0;
                if (m == 0) {
                    stage[n * n] = cn * f;
                } else {
                    stage[n * n + 2 * m - 1] = cn * f;
                    stage[n * n + 2 * m] = cn * f;
                }
                c2 = c1;
                c1 = cn;
            }
        }
    }
};

template <int P>
__device__ inline void coarse_s2_body(const Geo &g, int level, const double *__restrict__ psi,
                                      double *__restrict__ phic, int64_t blk, double *sL)
{
    constexpr int NT = (P + 1) * (P + 1);
    constexpr ScaledRegular<P> SR{};
    const int side = 1 << (level - 1), sh = g.L - level;
    const int Hh = 1 << sh;  // W / 2 = 2^(L-l)
    const int64_t orbits = (int64_t)Hh * Hh * Hh, Ml = (int64_t)side * side * side;
    const int C = coarse_cells_per_block(orbits);
    int64_t cell0, o0;
    if (C > 1) {
        cell0 = blk * C;
        o0 = 0;
    } else {
        const int64_t chunks = orbits / kCoarseThreads;
        cell0 = blk / chunks;
        o0 = (blk - cell0 * chunks) * kCoarseThreads;
    }
    for (int e = threadIdx.x; e < C * NT; e += blockDim.x) {
        const int k = e / C, c = e - k * C;
        sL[c * NT + k] = cell0 + c < Ml ? psi[(int64_t)k * Ml + cell0 + c] * SR.stage[k] : 0.0;
    }
    __syncthreads();
    const int cl = C > 1 ? (int)(threadIdx.x / orbits) : 0;
    const int64_t cell = cell0 + cl;
    if (cell >= Ml) return;
    // orbit b: its low three bits are the parities of (bx, by, bz), so for each
    // reflection eight consecutive lanes write the eight sites of one fine cell
    // (64 contiguous bytes) and a wave writes eight z-consecutive fine cells
    const int b = (int)(C > 1 ? threadIdx.x - cl * orbits : o0 + threadIdx.x);
    const int h2 = Hh >> 1, q = b >> 3;
    const int bx = 2 * (q / (h2 * h2)) + ((b >> 2) & 1), by = 2 * ((q / h2) % h2) + ((b >> 1) & 1),
              bz = 2 * (q % h2) + (b & 1);
    const int cx = (int)(cell / ((int64_t)side * side)), cy = (int)((cell / side) % side), cz = (int)(cell % side);
    const double x = (bx + 0.5) * g.h, y = (by + 0.5) * g.h, z = (bz + 0.5) * g.h;
    const double nr2 = -(x * x + y * y + z * z);
    const double *L = sL + cl * NT;
    // the orbit's eight sites
    const int W = 2 * Hh;
    int64_t at[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int fx = (u >> 2) & 1, fy = (u >> 1) & 1, fz = u & 1;  // 1: the reflected side
        const int i = cx * W + Hh + (fx ? -1 - bx : bx), j = cy * W + Hh + (fy ? -1 - by : by),
                  k = cz * W + Hh + (fz ? -1 - bz : bz);
        at[u] = s2_site(g.nc, i, j, k);
    }
    // class sums S[A][B][C]: A = (n + m) & 1, B = m & 1, C = 0 real / 1 imaginary part
    double S[2][2][2] = {};
    {  // m = 0 column
        double q2 = 1.0, q1 = z;
        S[0][0][0] = L[0];
        if (P >= 1) S[1][0][0] = L[slot0(1)] * z;
#pragma unroll
        for (int nn = 2; nn <= P; ++nn) {
            const double qn = fma(SR.g[nn][0] * z, q1, nr2 * q2);
            S[nn & 1][0][0] = fma(L[slot0(nn)], qn, S[nn & 1][0][0]);
            q2 = q1;
            q1 = qn;
        }
    }
    double dr = 1.0, di = 0.0;
#pragma unroll
    for (int m = 1; m <= P; ++m) {
        const double f = -0.5 / m;
        const double ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        double ar = dr, ai = di;
        const int B = m & 1;
        S[0][B][0] = fma(L[slot_re(m, m)], ar, S[0][B][0]);  // n = m: n + m even
        S[0][B][1] = fma(L[slot_im(m, m)], ai, S[0][B][1]);
        if (m + 1 <= P) {
            double br = z * ar, bi = z * ai;
            S[1][B][0] = fma(L[slot_re(m + 1, m)], br, S[1][B][0]);
            S[1][B][1] = fma(L[slot_im(m + 1, m)], bi, S[1][B][1]);
#pragma unroll
            for (int nn = m + 2; nn <= P; ++nn) {
                const double gz = SR.g[nn][m] * z;
                const double cr = fma(gz, br, nr2 * ar), ci = fma(gz, bi, nr2 * ai);
                const int A = (nn + m) & 1;
                S[A][B][0] = fma(L[slot_re(nn, m)], cr, S[A][B][0]);
                S[A][B][1] = fma(L[slot_im(nn, m)], ci, S[A][B][1]);
                ar = br;
                ai = bi;
                br = cr;
                bi = ci;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int fx = (u >> 2) & 1, fy = (u >> 1) & 1, fz = u & 1;
        double acc = 0.0;
#pragma unroll
        for (int A = 0; A < 2; ++A)
#pragma unroll
            for (int B = 0; B < 2; ++B) {
                const double sz = (fz && A) ? -1.0 : 1.0;
                const double sre = sz * ((fx && B) ? -1.0 : 1.0);
                const double sim = sz * ((fx && !B) ? -1.0 : 1.0) * (fy ? -1.0 : 1.0);
                acc += sre * S[A][B][0] + sim * S[A][B][1];
            }
        phic[at[u]] = acc;
    }
}

// blocks of the orbit kernel for one level of a 2x2x2 lattice with fine-cell count M
__host__ __device__ inline int64_t coarse_s2_blocks(int L, int level)
{
    const int sh = L - level;
    const int64_t orbits = (int64_t)1 << (3 * sh), Ml = (int64_t)1 << (3 * (level - 1));
    const int C = coarse_cells_per_block(orbits);
    return C > 1 ? (Ml + C - 1) / C : Ml * (orbits / kCoarseThreads);
}

// blocks of the orbit kernel for all coarse levels lstart .. L-1 of a 2x2x2
// lattice in one launch, level L-1 first
__host__ __device__ inline int64_t coarse_s2_all_blocks(int L, int lstart)
{
    int64_t b = 0;
    for (int l = L - 1; l >= lstart; --l) b += coarse_s2_blocks(L, l);
    return b;
}

// block blk of that launch: its level, and blk becomes the block within the level
__device__ inline int coarse_s2_level_of(int L, int lstart, int64_t &blk)
{
    int l = L - 1;
    for (; l > lstart; --l) {
        const int64_t nb = coarse_s2_blocks(L, l);
        if (blk < nb) break;
        blk -= nb;
    }
    return l;
}

// LDS of an orbit-kernel block: the most cells per block any level has (its finest, 8 orbits per cell)
inline size_t coarse_s2_shm(int p) { return sizeof(double) * (p + 1) * (p + 1) * coarse_cells_per_block(8); }

// every coarse level in one launch, level l into per-site array L-1-l
template <int P>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_s2(Geo g, double *const *__restrict__ psi_lv,
                                                   double *__restrict__ phic)
{
    extern __shared__ double sL[];
    int64_t blk = blockIdx.x;
    const int level = coarse_s2_level_of(g.L, g.lstart, blk);
    const int64_t ns = (int64_t)g.n * g.n * g.n;
    coarse_s2_body<P>(g, level, psi_lv[level], phic + (int64_t)(g.L - 1 - level) * ns, blk, sL);
}

void launch_coarse_sites(fmmkmc_ctx *c, const Geo &g)
{
    if (!c->per_level || !c->phicoarse) return;  // no coarser level with an interaction list
    const int lstart = g.lstart;
    if (c->s2) {
        FMMKMC_DISPATCH_P(c->p, launch_shm(c, "coarse_s2", k_coarse_s2<P_>,
                                           dim3((unsigned)coarse_s2_all_blocks(g.L, lstart)), dim3(kCoarseThreads),
                                           coarse_s2_shm(c->p), g, (double *const *)c->d_psi_ptrs, c->phicoarse));
    } else {
        const int64_t ns = (int64_t)c->lat_n * c->lat_n * c->lat_n;
        FMMKMC_DISPATCH_P(c->p, launch(c, "coarse_sites", k_coarse_sites<P_>, dim3((unsigned)((ns + 255) / 256)),
                                       dim3(256), g, (double *const *)c->d_psi_ptrs, 0, c->phicoarse));
    }
}

// ---- per-slot gather (lattice) ---------------------------------------------
// Charges are taken in rank order (site order), TCH per block; their packed
// coordinates, charge, phi_occ and caller index are staged in LDS once, so a
// slot needs a single gather: phi at the target site (NaN if occupied).  The
// F table is stored by rank, so its reads are contiguous; dU and mask go to
// the caller's [charge][hop] layout (K contiguous entries per charge).
constexpr int TCH = 64;   // charges per block (the single-context default)
constexpr int SLOTB = 4;  // slots per lane whose loads are in flight together

template <int TC>
__device__ __forceinline__ void slot_body(int64_t blk, Geo g, int64_t N, uint32_t K, uint32_t kmul,
                                          const int32_t *__restrict__ offs_, const int32_t *__restrict__ order_,
                                          const int32_t *__restrict__ ijk_r_, const double *__restrict__ q_r_,
                                          const double *__restrict__ phi_r_, const double *__restrict__ phisite_,
                                          const double *__restrict__ F_, const double *__restrict__ Fhop_,
                                          int s2, double *__restrict__ dU_, uint8_t *__restrict__ mask_)
{
    const auto offs = as_global(offs_), order = as_global(order_), ijk_r = as_global(ijk_r_);
    const auto q_r = as_global(q_r_), phi_r = as_global(phi_r_), phisite = as_global(phisite_), F = as_global(F_);
    const auto dU = as_global(dU_);
    const auto mask = as_global(mask_);
    __shared__ int32_t soff[3 * kMaxHops];
    __shared__ double sfhop[kMaxHops], sfield[kMaxHops];
    __shared__ int32_t s_ijk[TC], s_ord[TC];
    __shared__ double s_q[TC], s_phi[TC];
    const int64_t r0 = blk * TC;
    const int nloc = (int)((N - r0) < TC ? (N - r0) : TC);
    for (uint32_t e = threadIdx.x; e < 3 * K; e += blockDim.x) soff[e] = offs[e];
    const bool per_charge = g.periodic && F_ != nullptr;  // else a per-hop correction
    for (uint32_t e = threadIdx.x; e < K; e += blockDim.x) {
        double v = 0.0;
        if (!g.periodic) {
            const double ox = offs[3 * e], oy = offs[3 * e + 1], oz = offs[3 * e + 2];
            v = -1.0 / (g.h * sqrt(ox * ox + oy * oy + oz * oz));
        } else if (!per_charge) {
            v = Fhop_[e];
        }
        sfhop[e] = v;
        sfield[e] = field_work(g, g.h * offs[3 * e], g.h * offs[3 * e + 1], g.h * offs[3 * e + 2]);
    }
    if ((int)threadIdx.x < nloc) {
        const int64_t r = r0 + threadIdx.x;
        s_ijk[threadIdx.x] = ijk_r[r];
        s_ord[threadIdx.x] = order[r];
        s_q[threadIdx.x] = q_r[r];
        s_phi[threadIdx.x] = phi_r[r];
    }
    __syncthreads();
    const uint32_t total = (uint32_t)nloc * K;
    const int n = g.n, nc = g.nc;
    const double nanv = __builtin_nan("");
    for (uint32_t e0 = threadIdx.x; e0 < total; e0 += SLOTB * blockDim.x) {
        double v[SLOTB], f[SLOTB];
        uint32_t lc[SLOTB], kk[SLOTB];
#pragma unroll
        for (int b = 0; b < SLOTB; ++b) {
            const uint32_t e = e0 + b * blockDim.x;
            v[b] = nanv;
            f[b] = 0.0;
            lc[b] = 0;
            kk[b] = 0;
            if (e >= total) continue;
            uint32_t c = __umulhi(e, kmul), k = e - c * K;
            if (k >= K) {
                ++c;
                k -= K;
            }
            lc[b] = c;
            kk[b] = k;
            const int32_t pk = s_ijk[c];
            int ti = (pk >> 20) + soff[3 * k], tj = ((pk >> 10) & 1023) + soff[3 * k + 1],
                tk = (pk & 1023) + soff[3 * k + 2];
            bool inside = true;
            if (g.periodic) {
                ti += ti < 0 ? n : (ti >= n ? -n : 0);
                tj += tj < 0 ? n : (tj >= n ? -n : 0);
                tk += tk < 0 ? n : (tk >= n ? -n : 0);
            } else {
                inside = ti >= 0 && ti < n && tj >= 0 && tj < n && tk >= 0 && tk < n;
            }
            if (inside) {
                const int64_t pt = s2 ? ((((int64_t)(ti >> 1) * nc + (tj >> 1)) * nc + (tk >> 1)) * 8 +
                                         ((ti & 1) * 4 + (tj & 1) * 2 + (tk & 1)))
                                      : (((int64_t)ti * n + tj) * n + tk);
                v[b] = phisite[pt];
            }
            if (per_charge) f[b] = F[r0 * K + e];
        }
#pragma unroll
        for (int b = 0; b < SLOTB; ++b) {
            const uint32_t e = e0 + b * blockDim.x;
            if (e >= total) continue;
            const uint32_t c = lc[b], k = kk[b];
            const double qi = s_q[c];
            const double corr = per_charge ? f[b] : sfhop[k];
            const bool valid = !__builtin_isnan(v[b]);
            const double out = valid ? qi * (v[b] - s_phi[c] + sfield[k]) + qi * qi * corr : nanv;
            const int64_t o = (int64_t)s_ord[c] * K + k;
            dU[o] = out;
            if (mask) mask[o] = valid ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_slot_lattice(Geo g, int64_t N, uint32_t K, uint32_t kmul,
                                                      const int32_t *__restrict__ offs,
                                                      const int32_t *__restrict__ order,
                                                      const int32_t *__restrict__ ijk_r, const double *__restrict__ q_r,
                                                      const double *__restrict__ phi_r,
                                                      const double *__restrict__ phisite,
                                                      const double *__restrict__ F, const double *__restrict__ Fhop,
                                                      int s2, double *__restrict__ dU, uint8_t *__restrict__ mask)
{
    slot_body<TCH>(blockIdx.x, g, N, K, kmul, offs, order, ijk_r, q_r, phi_r, phisite, F, Fhop, s2, dU, mask);
}

void launch_slot_lattice(fmmkmc_ctx *c, const Geo &g, int K, double *dU, uint8_t *mask)
{
    const uint32_t kmul = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)K);
    launch(c, "slot_lattice", k_slot_lattice, dim3((unsigned)((c->N + TCH - 1) / TCH)), dim3(256), g, c->N,
           (uint32_t)K, kmul, c->d_offsets, c->order, c->ijk_r, c->q_r, c->phi_r, c->phisite,
           c->self_exact ? nullptr : c->F, c->Fhop, c->s2 ? 1 : 0, dU, mask);
}

// exact self-image option: the per-hop change G_self - G(h offsets[k]) (the
// Ewald sum of ewald.hpp), one lane per hop
__global__ void k_self_hops(int K, const int32_t *__restrict__ offs, double h, double a, double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    out[k] = periodic_self_change(a, h * offs[3 * k], h * offs[3 * k + 1], h * offs[3 * k + 2]);
}

void launch_self_hops(fmmkmc_ctx *c, int K)
{
    launch(c, "self_hops", k_self_hops, dim3(1), dim3(64), K, c->d_offsets, c->h, c->a, c->Fhop);
}

// ---- far-field helpers (LDS-tiled matrix-vector products with R) ----------

constexpr int SB = 8;  // items per block (2 LDS rows of (p+1)^2 doubles each, <= 37 KB)

// sigma(s) = B(s, s) with B(y, x) = L2P of R K1(x) at y: the V_inf field at a
// site due to a unit charge at the same site, for every lattice site.
__global__ __launch_bounds__(256) void k_sigma_sites(Geo g, int p, const double *__restrict__ R,
                                                     double *__restrict__ sigma)
{
    const int nt = nterms(p);
    extern __shared__ double sm[];
    double *Kv = sm, *Wv = sm + SB * nt;
    const int n = g.n;
    const int64_t ns = (int64_t)n * n * n;
    const int64_t s0 = (int64_t)blockIdx.x * SB;
    if (threadIdx.x < SB) {
        const int64_t s = s0 + threadIdx.x;
        if (s < ns) {
            const int si = (int)(s / ((int64_t)n * n)), sj = (int)((s / n) % n), sk = (int)(s % n);
            unit_multipole_and_weights(p, (si + 0.5) * g.h - 0.5 * g.a, (sj + 0.5) * g.h - 0.5 * g.a,
                                       (sk + 0.5) * g.h - 0.5 * g.a, Kv + threadIdx.x * nt, Wv + threadIdx.x * nt);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SB * nt; e += blockDim.x) {
        const int b = e / nt, k = e % nt;
        if (s0 + b >= ns) continue;
        double acc = 0.0;
        for (int m = 0; m < nt; ++m) acc += R[(int64_t)m * nt + k] * Kv[b * nt + m];
        Wv[b * nt + k] *= acc;
    }
    __syncthreads();
    if (threadIdx.x < SB && s0 + threadIdx.x < ns) {
        double acc = 0.0;
        for (int k = 0; k < nt; ++k) acc += Wv[threadIdx.x * nt + k];
        sigma[s0 + threadIdx.x] = acc;
    }
}

// F[i][k] for the lattice fast path (periodic): the q^2-terms of a hop,
//   -sum_{nu in V_box} 1/|t - r - a nu| + C_box / a + 1/2 (sigma(t) + sigma(r)) - B(t, r)
// for charge i at site r and its wrapped target t (charges given by rank).
__global__ __launch_bounds__(256) void k_f_rows(Geo g, int p, int64_t count, const int32_t *__restrict__ order,
                                                int64_t first, int K, const int32_t *__restrict__ offs,
                                                const int32_t *__restrict__ site, const double *__restrict__ R,
                                                const double *__restrict__ sigma, double *__restrict__ F)
{
    const int nt = nterms(p);
    extern __shared__ double sm[];
    double *Kv = sm, *Wv = sm + SB * nt;
    const int n = g.n;
    const int64_t c0 = (int64_t)blockIdx.x * SB;
    if (threadIdx.x < SB && c0 + threadIdx.x < count) {
        const int64_t i = order[first + c0 + threadIdx.x];
        const int s = site[i];
        const int si = s / (n * n), sj = (s / n) % n, sk = s % n;
        unit_multipole_and_weights(p, (si + 0.5) * g.h - 0.5 * g.a, (sj + 0.5) * g.h - 0.5 * g.a,
                                   (sk + 0.5) * g.h - 0.5 * g.a, Kv + threadIdx.x * nt, Wv + threadIdx.x * nt);
    }
    __syncthreads();
    // Wv <- R K1(r) (the V_inf local expansion of a unit charge at r)
    for (int e = threadIdx.x; e < SB * nt; e += blockDim.x) {
        const int b = e / nt, k = e % nt;
        if (c0 + b >= count) continue;
        double acc = 0.0;
        for (int m = 0; m < nt; ++m) acc += R[(int64_t)m * nt + k] * Kv[b * nt + m];
        Wv[b * nt + k] = acc;
    }
    __syncthreads();
    const double cbox = (6.0 + 8.0 / sqrt(3.0) + 12.0 / sqrt(2.0)) / g.a;
    for (int e = threadIdx.x; e < SB * K; e += blockDim.x) {
        const int b = e / K, k = e % K;
        if (c0 + b >= count) continue;
        const int64_t rk = first + c0 + b, i = order[rk];
        const int s = site[i];
        const int si = s / (n * n), sj = (s / n) % n, sk = s % n;
        const int ti = posmod(si + offs[3 * k], n), tj = posmod(sj + offs[3 * k + 1], n),
                  tk = posmod(sk + offs[3 * k + 2], n);
        const double rx = (si + 0.5) * g.h, ry = (sj + 0.5) * g.h, rz = (sk + 0.5) * g.h;
        const double tx = (ti + 0.5) * g.h, ty = (tj + 0.5) * g.h, tz = (tk + 0.5) * g.h;
        double self = 0.0;
        for (int a0 = -1; a0 <= 1; ++a0)
            for (int a1 = -1; a1 <= 1; ++a1)
                for (int a2 = -1; a2 <= 1; ++a2) {
                    const double d0 = tx - rx - g.a * a0, d1 = ty - ry - g.a * a1, d2 = tz - rz - g.a * a2;
                    self += 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                }
        const double B = l2p_runtime(p, Wv + b * nt, 1, tx - 0.5 * g.a, ty - 0.5 * g.a, tz - 0.5 * g.a);
        const int64_t ts = ((int64_t)ti * n + tj) * n + tk;
        F[rk * K + k] = -self + cbox + 0.5 * (sigma[ts] + sigma[s]) - B;
    }
}

// F row of one charge (after an accept), in two launches so that no block
// walks a long chain of dependent loads:
//   1. w = R K1(r), the V_inf local expansion of a unit charge at the charge's
//      new site r: kFrowRows rows of w per block, each row split over 16 lanes;
//   2. one 64-lane block per hop k: the weights W(t_k) of its wrapped target,
//      B_k = W(t_k) . w, the 27 self distances, and F[rank][k].
constexpr int kFrowRows = 16;

__host__ __device__ constexpr int frow_w_blocks(int nt)
{
    return (nt + kFrowRows - 1) / kFrowRows;
}

__device__ __forceinline__ void frow_w_body(int blk, Geo g, int p, int64_t s_site, const double *__restrict__ R,
                                            double *__restrict__ w)
{
    const int nt = nterms(p);
    __shared__ double K1[(kMaxOrder + 1) * (kMaxOrder + 1)], Wd[(kMaxOrder + 1) * (kMaxOrder + 1)];
    __shared__ double red[256];
    const int n = g.n, s = (int)s_site;
    const int si = s / (n * n), sj = (s / n) % n, sk = s % n;
    const double c = 0.5 * g.a;
    const int tid = threadIdx.x;
    if (tid <= p) harmonics_column(p, tid, (si + 0.5) * g.h - c, (sj + 0.5) * g.h - c, (sk + 0.5) * g.h - c, K1, Wd);
    __syncthreads();
    const int lr = tid & 15, ls = tid >> 4, row = blk * kFrowRows + lr;
    double acc = 0.0;
    if (row < nt) {
        // four independent loads in flight
        double a4[4] = {};
        int m = ls;
        for (; m + 48 < nt; m += 64) {
            double r4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) r4[u] = R[(int64_t)(m + 16 * u) * nt + row];
#pragma unroll
            for (int u = 0; u < 4; ++u) a4[u] += r4[u] * K1[m + 16 * u];
        }
        for (; m < nt; m += 16) a4[0] += R[(int64_t)m * nt + row] * K1[m];
        acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    red[tid] = acc;
    __syncthreads();
    if (ls == 0 && row < nt) {
        double sum = 0.0;
        for (int t = 0; t < 16; ++t) sum += red[t * 16 + lr];
        w[row] = sum;
    }
}

__device__ __forceinline__ void frow_b_body(int k, Geo g, int p, int64_t rank, int64_t s_site, int K,
                                            const int32_t *__restrict__ offs, const double *__restrict__ w,
                                            const double *__restrict__ sigma, double *__restrict__ F)
{
    const int nt = nterms(p);
    __shared__ double Wt[(kMaxOrder + 1) * (kMaxOrder + 1)];
    __shared__ double red[64], selfv[27];
    const int n = g.n, s = (int)s_site;
    const int si = s / (n * n), sj = (s / n) % n, sk = s % n;
    const double c = 0.5 * g.a;
    const int tid = threadIdx.x;
    const int ti = posmod(si + offs[3 * k], n), tj = posmod(sj + offs[3 * k + 1], n),
              tk = posmod(sk + offs[3 * k + 2], n);
    const double tx = (ti + 0.5) * g.h, ty = (tj + 0.5) * g.h, tz = (tk + 0.5) * g.h;
    if (tid <= p) harmonics_column(p, tid, tx - c, ty - c, tz - c, nullptr, Wt);
    if (tid >= 32 && tid < 32 + 27) {
        const int nu = tid - 32;
        const double d0 = tx - (si + 0.5) * g.h - g.a * (nu / 9 - 1),
                     d1 = ty - (sj + 0.5) * g.h - g.a * ((nu / 3) % 3 - 1),
                     d2 = tz - (sk + 0.5) * g.h - g.a * (nu % 3 - 1);
        selfv[nu] = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    __syncthreads();
    double b = 0.0;
    for (int m = tid; m < nt; m += 64) b += Wt[m] * w[m];
    red[tid] = b;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        double self = 0.0;
        for (int nu = 0; nu < 27; ++nu) self += selfv[nu];
        const double cbox = (6.0 + 8.0 / sqrt(3.0) + 12.0 / sqrt(2.0)) / g.a;
        const int64_t ts = ((int64_t)ti * n + tj) * n + tk;
        F[rank * K + k] = -self + cbox + 0.5 * (sigma[ts] + sigma[s]) - red[0];
    }
}

__global__ __launch_bounds__(256) void k_frow_w(Geo g, int p, int64_t s_site, const double *__restrict__ R,
                                                double *__restrict__ w)
{
    frow_w_body(blockIdx.x, g, p, s_site, R, w);
}

__global__ __launch_bounds__(64) void k_frow_b(Geo g, int p, int64_t rank, int64_t s_site, int K,
                                               const int32_t *__restrict__ offs, const double *__restrict__ w,
                                               const double *__restrict__ sigma, double *__restrict__ F)
{
    frow_b_body(blockIdx.x, g, p, rank, s_site, K, offs, w, sigma, F);
}

void launch_sigma(fmmkmc_ctx *c, const Geo &g)
{
    const int64_t ns = (int64_t)c->lat_n * c->lat_n * c->lat_n;
    const size_t shm = sizeof(double) * 2 * SB * c->nt;
    launch_shm(c, "sigma_sites", k_sigma_sites, dim3((unsigned)((ns + SB - 1) / SB)), dim3(256), shm, g, c->p,
               c->far.R, c->far.sigma);
}

void launch_f_row1(fmmkmc_ctx *c, const Geo &g, int K, int64_t rank, int64_t site, hipStream_t st)
{
    launch_on(c, st, "f_row1", k_frow_w, dim3(frow_w_blocks(c->nt)), dim3(256), 0, g, c->p, site, c->far.R,
              c->frow_w);
    launch_on(c, st, "f_row1", k_frow_b, dim3(K), dim3(64), 0, g, c->p, rank, site, K, c->d_offsets, c->frow_w,
              c->far.sigma, c->F);
}

void launch_f_rows(fmmkmc_ctx *c, const Geo &g, int64_t count, int K, int64_t first)
{
    const size_t shm = sizeof(double) * 2 * SB * c->nt;
    launch_shm(c, "f_rows", k_f_rows, dim3((unsigned)((count + SB - 1) / SB)), dim3(256), shm, g, c->p, count,
               c->order, first, K, c->d_offsets, c->site, c->far.R, c->far.sigma, c->F);
}

// ---- dU of one move (accept step), one block, FP64 ----------------------------

__device__ inline double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Same terms as a proposal (header of this file), recomputed for the accepted
// move (footnote to Sec. 3.1), always from the FP64 local expansions.  Four
// blocks work on independent parts and each writes one partial sum:
//   0: q (Psi(t) - Psi(r)) from the fine-level local expansions, and the self terms
//   1: q times the near field at t,  2: minus q times the near field at r
//      (the moving charge itself left out)
//   3: the far-field change q dW.H + 1/2 q dW^T R dK (periodic; else 0)
__device__ __forceinline__ void move_dU_body(int part_id, Geo g, int p, int64_t M, int64_t i, double tx, double ty,
                                             double tz, const double *__restrict__ psi,
                                             const double *__restrict__ x, const double *__restrict__ y,
                                             const double *__restrict__ z, const double *__restrict__ q,
                                             const int32_t *__restrict__ cnt, const int32_t *__restrict__ slots,
                                             const double *__restrict__ R, const double *__restrict__ H,
                                             double *__restrict__ out, double *const *__restrict__ psi_lv)
{
    const int nt = nterms(p);
    extern __shared__ double sm[];
    double *red = sm;  // 256
    double *Wa = sm + 256, *Wb = Wa + nt, *Ka = Wb + nt, *Kb = Ka + nt;
    __shared__ int32_t s_cnt[27];
    __shared__ int64_t s_cell[27];
    __shared__ double s_shift[27][3];
    const double rx = x[i], ry = y[i], rz = z[i], qi = q[i];
    const int tcx = fine_coord(tx, g.w, g.nc), tcy = fine_coord(ty, g.w, g.nc), tcz = fine_coord(tz, g.w, g.nc);
    const int rcx = fine_coord(rx, g.w, g.nc), rcy = fine_coord(ry, g.w, g.nc), rcz = fine_coord(rz, g.w, g.nc);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    double part = 0.0;
    if (part_id == 0) {
        // q (Psi(t) - Psi(r)): the fine level, and in per-level mode every coarser
        // level too, each about the centre of the level's cell holding t or r.
        // Harmonics of every (level, endpoint, column m) at once, one lane each,
        // then the dot products over the block (every level's loads independent).
        const int l0 = g.per_level ? g.lstart : g.L, nlev = g.L - l0 + 1;
        double *Wl = sm + 256;  // [level][endpoint][nt]
        // per level: its expansions, cell count and the cells holding t and r
        // (the level pointers read once, beside the harmonics below)
        __shared__ const double *s_pl[kMaxLevels + 1];
        __shared__ int64_t s_ml[kMaxLevels + 1], s_tc[kMaxLevels + 1], s_rc[kMaxLevels + 1];
        if ((int)threadIdx.x < nlev) {
            const int li = threadIdx.x, l = l0 + li, side = 1 << (l - 1), sh = g.L - l;
            s_pl[li] = l == g.L ? psi : psi_lv[l];
            s_ml[li] = (int64_t)side * side * side;
            s_tc[li] = cell_id(side, tcx >> sh, tcy >> sh, tcz >> sh);
            s_rc[li] = cell_id(side, rcx >> sh, rcy >> sh, rcz >> sh);
        }
        for (int task = threadIdx.x; task < nlev * 2 * (p + 1); task += blockDim.x) {
            const int li = task / (2 * (p + 1)), e = (task / (p + 1)) & 1, m = task % (p + 1);
            const int l = l0 + li, side = 1 << (l - 1), sh = g.L - l;
            const double w = g.a / side;
            const int cx = (e ? rcx : tcx) >> sh, cy = (e ? rcy : tcy) >> sh, cz = (e ? rcz : tcz) >> sh;
            harmonics_column(p, m, (e ? rx : tx) - (cx + 0.5) * w, (e ? ry : ty) - (cy + 0.5) * w,
                             (e ? rz : tz) - (cz + 0.5) * w, nullptr, Wl + (int64_t)(2 * li + e) * nt);
        }
        __syncthreads();
        // (level, coefficient) pairs over the block, four per thread in flight
        const int ne = nlev * nt;
        for (int e0 = threadIdx.x; e0 < ne; e0 += 4 * blockDim.x) {
            double tv[4], rv[4], wt[4], wr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * (int)blockDim.x;
                tv[u] = rv[u] = wt[u] = wr[u] = 0.0;
                if (e < ne) {
                    const int li = e / nt, k = e - li * nt;
                    const double *pl = s_pl[li] + (int64_t)k * s_ml[li];
                    tv[u] = pl[s_tc[li]];
                    rv[u] = pl[s_rc[li]];
                    wt[u] = Wl[(int64_t)(2 * li) * nt + k];
                    wr[u] = Wl[(int64_t)(2 * li + 1) * nt + k];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (e0 + u * (int)blockDim.x < ne) part += qi * (tv[u] * wt[u] - rv[u] * wr[u]);
        }
        if (threadIdx.x == 0) part += qi * field_work(g, tx - rx, ty - ry, tz - rz);  // uniform field
        // self terms: one copy nu of the old position per lane, or the exact
        // self-image change with its Ewald terms split over the block
        if (g.periodic && g.self_exact) {
            part += qi * qi * periodic_self_change_share(g.a, tx - rx, ty - ry, tz - rz, threadIdx.x, blockDim.x);
        } else if (g.periodic) {
            if (threadIdx.x < 27) {
                const int nu = threadIdx.x;
                const double d0 = tx - rx - g.a * (nu / 9 - 1), d1 = ty - ry - g.a * ((nu / 3) % 3 - 1),
                             d2 = tz - rz - g.a * (nu % 3 - 1);
                part -= qi * qi / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            }
            if (threadIdx.x == 0) part += qi * qi * (6.0 + 8.0 / sqrt(3.0) + 12.0 / sqrt(2.0)) / g.a;
        } else if (threadIdx.x == 0) {
            const double d0 = tx - rx, d1 = ty - ry, d2 = tz - rz;
            part -= qi * qi / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
    } else if (part_id <= 2) {
        // near field of one endpoint: the neighbour cells' counts first, then one lane per (cell, slot)
        const int e = part_id - 1;  // 0: target, 1: old position
        const int bx = e ? rcx : tcx, by = e ? rcy : tcy, bz = e ? rcz : tcz;
        if (threadIdx.x < 27) {
            const int nb = threadIdx.x;
            int ax = bx + nb / 9 - 1, ay = by + (nb / 3) % 3 - 1, az = bz + nb % 3 - 1;
            double shx = 0, shy = 0, shz = 0;
            bool ok = true;
            if (ax < 0 || ax >= g.nc || ay < 0 || ay >= g.nc || az < 0 || az >= g.nc) {
                ok = g.periodic != 0;
                shx = g.a * floordiv(ax, g.nc);
                shy = g.a * floordiv(ay, g.nc);
                shz = g.a * floordiv(az, g.nc);
                ax = posmod(ax, g.nc);
                ay = posmod(ay, g.nc);
                az = posmod(az, g.nc);
            }
            const int64_t nbc = cell_id(g.nc, ax, ay, az);
            s_cell[nb] = nbc;
            s_cnt[nb] = ok ? cnt[nbc] : 0;
            s_shift[nb][0] = shx;
            s_shift[nb][1] = shy;
            s_shift[nb][2] = shz;
        }
        __syncthreads();
        const double px = e ? rx : tx, py = e ? ry : ty, pz = e ? rz : tz;
        for (int it = threadIdx.x; it < 27 * g.cap; it += blockDim.x) {
            const int nb = it / g.cap, sl = it - nb * g.cap;
            if (sl >= s_cnt[nb]) continue;
            const int j = slots[s_cell[nb] * g.cap + sl];
            const double shx = s_shift[nb][0], shy = s_shift[nb][1], shz = s_shift[nb][2];
            if (e == 1 && j == i && shx == 0 && shy == 0 && shz == 0) continue;
            const double d0 = px - (x[j] + shx), d1 = py - (y[j] + shy), d2 = pz - (z[j] + shz);
            const double v = qi * q[j] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            part += e ? -v : v;
        }
    } else if (g.periodic) {
        // q dW.H + 1/2 q dW^T R dK with dK = q (K1(t) - K1(r)), dW = W(t) - W(r),
        // harmonics about the box centre; the bilinear form over all (m, k) pairs
        const double c = 0.5 * g.a;
        double *Wt = Wa, *Wr = Wb, *Kt = Ka, *Kr = Kb;
        if (ln <= p) {
            if (wv == 0)
                harmonics_column(p, ln, tx - c, ty - c, tz - c, Kt, Wt);
            else if (wv == 1)
                harmonics_column(p, ln, rx - c, ry - c, rz - c, Kr, Wr);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nt; k += blockDim.x) {
            Kt[k] = qi * (Kt[k] - Kr[k]);
            Wt[k] = Wt[k] - Wr[k];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nt; k += blockDim.x) part += qi * Wt[k] * H[k];
        // dW^T R dK: lane (k, group) runs down column k of R over the rows m of
        // its group, so consecutive lanes read consecutive words and no lane
        // divides per element; four independent loads in flight per lane (the
        // quadratic term is part of the exact self-image change when that
        // option is on)
        if (!g.self_exact) {
            const int ng = (int)blockDim.x >= 2 * nt ? (int)blockDim.x / nt : 1;  // row groups
            for (int task = threadIdx.x; task < ng * nt; task += blockDim.x) {
                const int grp = task / nt, k = task - grp * nt;
                double a4[4] = {};
                int m = grp;
                for (; m + 3 * ng < nt; m += 4 * ng) {
                    double r4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) r4[u] = R[(int64_t)(m + u * ng) * nt + k];
#pragma unroll
                    for (int u = 0; u < 4; ++u) a4[u] += r4[u] * Kt[m + u * ng];
                }
                for (; m < nt; m += ng) a4[0] += R[(int64_t)m * nt + k] * Kt[m];
                part += 0.5 * qi * Wt[k] * ((a4[0] + a4[1]) + (a4[2] + a4[3]));
            }
        }
    }
    const double tot = block_sum(part, red);
    if (threadIdx.x == 0) out[part_id] = tot;
}

__global__ __launch_bounds__(256) void k_move_dU(Geo g, int p, int64_t M, int64_t i, double tx, double ty, double tz,
                                                 const double *__restrict__ psi, const double *__restrict__ x,
                                                 const double *__restrict__ y, const double *__restrict__ z,
                                                 const double *__restrict__ q, const int32_t *__restrict__ cnt,
                                                 const int32_t *__restrict__ slots, const double *__restrict__ R,
                                                 const double *__restrict__ H, double *__restrict__ out, int part0,
                                                 double *const *__restrict__ psi_lv)
{
    move_dU_body(part0 + (int)blockIdx.x, g, p, M, i, tx, ty, tz, psi, x, y, z, q, cnt, slots, R, H, out, psi_lv);
}

// LDS of a move-dU block: 256 reduction slots, then the four far-field vectors
// or the harmonics of every level and endpoint (per-level mode)
size_t move_dU_shm(int nt, int nlev) { return sizeof(double) * ((size_t)std::max(4, 2 * nlev) * nt + 256); }

void launch_move_dU(fmmkmc_ctx *c, const Geo &g, int64_t i, const double t[3], double *out, hipStream_t st,
                    int part0, int nparts)
{
    const size_t shm = move_dU_shm(c->nt, g.per_level ? g.L - g.lstart + 1 : 1);
    launch_on(c, st ? st : c->stream, part0 == 0 ? "move_dU" : "move_dU_side", k_move_dU, dim3(nparts), dim3(256),
              shm, g, c->p, c->M, i, t[0], t[1], t[2], c->psi_lv[c->L], c->x, c->y, c->z, c->q, c->cell_cnt,
              c->cell_slots, c->far.R, c->far.H, out, part0, (double *const *)c->d_psi_ptrs);
}

// ---- generic proposals ----------------------------------------------------

// wrap / validate targets; status: 0 ok, 1 outside (free), 2 coincident, 3 not used
__global__ __launch_bounds__(256) void k_prepare_targets(Geo g, int64_t S, const double *__restrict__ tgt,
                                                         const int32_t *__restrict__ use,
                                                         const double *__restrict__ x, const double *__restrict__ y,
                                                         const double *__restrict__ z,
                                                         const int32_t *__restrict__ cnt,
                                                         const int32_t *__restrict__ slots, double *__restrict__ tw,
                                                         int32_t *__restrict__ status, int32_t *__restrict__ flags)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double t[3] = {tgt[3 * s], tgt[3 * s + 1], tgt[3 * s + 2]};
    int st = (use && !use[s]) ? 3 : 0;
    for (int d = 0; d < 3 && st == 0; ++d) {
        if (g.periodic) {
            t[d] = wrap_coord(t[d], g.a);
        } else if (!(t[d] >= 0.0 && t[d] < g.a)) {
            st = 1;
        }
    }
    if (st == 0) {
        const int64_t cell = cell_id(g.nc, fine_coord(t[0], g.w, g.nc), fine_coord(t[1], g.w, g.nc),
                                     fine_coord(t[2], g.w, g.nc));
        for (int k = 0; k < cnt[cell]; ++k) {
            const int j = slots[cell * g.cap + k];
            if (x[j] == t[0] && y[j] == t[1] && z[j] == t[2]) st = 2;
        }
    } else {
        t[0] = t[1] = t[2] = 0.5 * g.a;  // harmless point for the later kernels
    }
    tw[3 * s] = t[0];
    tw[3 * s + 1] = t[1];
    tw[3 * s + 2] = t[2];
    status[s] = st;
    if (st == 1) atomicOr(flags, 1);
    if (st == 2) atomicOr(flags, 2);
}

// far-field change of each proposal: q (phi_inf(t) - phi_inf(r)) + 1/2 q (dphi(t) - dphi(r))
constexpr int SBF = 4;  // proposals per block (four LDS rows of (p+1)^2 doubles, <= 37 KB)

__global__ __launch_bounds__(256) void k_generic_far(Geo g, int p, int64_t S, const double *__restrict__ tw,
                                                     const int64_t *__restrict__ charge,
                                                     const double *__restrict__ x, const double *__restrict__ y,
                                                     const double *__restrict__ z, const double *__restrict__ q,
                                                     const double *__restrict__ R, const double *__restrict__ H,
                                                     double *__restrict__ far)
{
    const int nt = nterms(p);
    extern __shared__ double sm[];
    double *Kt = sm, *Wt = sm + SBF * nt, *Kr = sm + 2 * SBF * nt, *Wr = sm + 3 * SBF * nt;
    const int64_t s0 = (int64_t)blockIdx.x * SBF;
    const double c = 0.5 * g.a;
    const int b = threadIdx.x;
    // one lane per (proposal, endpoint, column m)
    for (int task = threadIdx.x; task < SBF * 2 * (p + 1); task += blockDim.x) {
        const int bb = task / (2 * (p + 1)), e = (task / (p + 1)) & 1, m = task % (p + 1);
        if (s0 + bb >= S) continue;
        const int64_t s = s0 + bb, i = charge[s];
        if (e == 0)
            harmonics_column(p, m, tw[3 * s] - c, tw[3 * s + 1] - c, tw[3 * s + 2] - c, Kt + bb * nt, Wt + bb * nt);
        else
            harmonics_column(p, m, x[i] - c, y[i] - c, z[i] - c, Kr + bb * nt, Wr + bb * nt);
    }
    __syncthreads();
    // Kt <- dK = q (K1(t) - K1(r)), Wt <- W(t) - W(r)
    for (int e = threadIdx.x; e < SBF * nt; e += blockDim.x) {
        const int bb = e / nt;
        if (s0 + bb >= S) continue;
        const double qi = q[charge[s0 + bb]];
        Kt[e] = qi * (Kt[e] - Kr[e]);
        Wt[e] = Wt[e] - Wr[e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SBF * nt; e += blockDim.x) {
        const int bb = e / nt, k = e % nt;
        if (s0 + bb >= S) continue;
        double dh = 0.0;
        // with the exact self-image option the quadratic term is not taken here
        if (!g.self_exact)
            for (int m = 0; m < nt; ++m) dh += R[(int64_t)m * nt + k] * Kt[bb * nt + m];
        const double qi = q[charge[s0 + bb]];
        Kr[e] = Wt[e] * qi * (H[k] + 0.5 * dh);
    }
    __syncthreads();
    if (b < SBF && s0 + b < S) {
        double acc = 0.0;
        for (int k = 0; k < nt; ++k) acc += Kr[b * nt + k];
        far[s0 + b] = acc;
    }
}

// dU = q (phi(t) - phi_occ(r)) + self terms + far
__global__ __launch_bounds__(256) void k_generic_combine(Geo g, int64_t S, const double *__restrict__ tw,
                                                         const int32_t *__restrict__ status,
                                                         const int64_t *__restrict__ charge,
                                                         const double *__restrict__ x, const double *__restrict__ y,
                                                         const double *__restrict__ z, const double *__restrict__ q,
                                                         const double *__restrict__ phit,
                                                         const double *__restrict__ phir,
                                                         const double *__restrict__ far, double *__restrict__ dU)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (status[s] != 0) {
        dU[s] = __builtin_nan("");
        return;
    }
    const int64_t i = charge[s];
    const double qi = q[i];
    const double tx = tw[3 * s], ty = tw[3 * s + 1], tz = tw[3 * s + 2];
    double d = qi * (phit[s] - phir[s] + field_work(g, tx - x[i], ty - y[i], tz - z[i]));
    if (g.periodic && g.self_exact) {
        d += qi * qi * periodic_self_change(g.a, tx - x[i], ty - y[i], tz - z[i]) + far[s];
    } else if (g.periodic) {
        double self = 0.0;
        for (int a0 = -1; a0 <= 1; ++a0)
            for (int a1 = -1; a1 <= 1; ++a1)
                for (int a2 = -1; a2 <= 1; ++a2) {
                    const double d0 = tx - x[i] - g.a * a0, d1 = ty - y[i] - g.a * a1, d2 = tz - z[i] - g.a * a2;
                    self += 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                }
        d += -qi * qi * self + qi * qi * (6.0 + 8.0 / sqrt(3.0) + 12.0 / sqrt(2.0)) / g.a + far[s];
    } else {
        const double d0 = tx - x[i], d1 = ty - y[i], d2 = tz - z[i];
        d -= qi * qi / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    }
    dU[s] = d;
}

// slot -> charge index from the CSR groups
__global__ void k_expand_groups(int64_t G, const int64_t *__restrict__ idx, const int64_t *__restrict__ offs,
                                int64_t *__restrict__ charge)
{
    const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= G) return;
    for (int64_t s = offs[gi]; s < offs[gi + 1]; ++s) charge[s] = idx[gi];
}

// propose_with_dats: slots (i, k) with k < C[T[i]] and M[i][k] != 0
__global__ void k_dats_select(int64_t N, int K, const int32_t *__restrict__ C, int ntypes,
                              const int32_t *__restrict__ T, const uint8_t *__restrict__ Mk,
                              int32_t *__restrict__ use, int32_t *__restrict__ flags)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * K) return;
    const int64_t i = t / K;
    const int k = (int)(t - i * K);
    const int ty = T[i];
    int u = 0;
    if (ty < 0 || ty >= ntypes) {
        atomicOr(flags, 4);
    } else {
        u = (k < C[ty] && Mk[t] != 0) ? 1 : 0;
    }
    use[t] = u;
}

void launch_generic(fmmkmc_ctx *c, const Geo &g, int64_t S, const double *tgt, const int64_t *charge, double *dU,
                    double *work, const int32_t *use)
{
    // work layout: tw[3S] phit[S] phir[S] far[S] status[S] (int32)
    double *tw = work, *phit = tw + 3 * S, *phir = phit + S, *far = phir + S;
    int32_t *status = (int32_t *)(far + S);
    dim3 grid((unsigned)((S + 255) / 256));
    launch(c, "prepare_targets", k_prepare_targets, grid, dim3(256), g, S, tgt, use, c->x, c->y, c->z,
           c->cell_cnt, c->cell_slots, tw, status, c->flags);
    launch_point_phi(c, g, S, tw, nullptr, nullptr, 0, phit, "point_phi");
    launch_point_phi(c, g, S, nullptr, charge, charge, 0, phir, "point_phi");
    if (g.periodic) {
        const size_t shm = sizeof(double) * 4 * SBF * c->nt;
        launch_shm(c, "generic_far", k_generic_far, dim3((unsigned)((S + SBF - 1) / SBF)), dim3(256), shm, g, c->p,
                   S, tw, charge, c->x, c->y, c->z, c->q, c->far.R, c->far.H, far);
    }
    launch(c, "generic_combine", k_generic_combine, grid, dim3(256), g, S, tw, status, charge, c->x, c->y, c->z,
           c->q, phit, phir, far, dU);
}

__global__ void k_div_index(int64_t S, int K, int64_t *__restrict__ charge)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) charge[s] = s / K;
}

void launch_div_index(fmmkmc_ctx *c, int64_t S, int K, int64_t *charge)
{
    launch(c, "div_index", k_div_index, dim3((unsigned)((S + 255) / 256)), dim3(256), S, K, charge);
}

void launch_expand_groups(fmmkmc_ctx *c, int64_t G, const int64_t *idx, const int64_t *offs, int64_t *charge)
{
    launch(c, "expand_groups", k_expand_groups, dim3((unsigned)((G + 255) / 256)), dim3(256), G, idx, offs, charge);
}

void launch_dats_select(fmmkmc_ctx *c, int64_t N, int K, const int32_t *C, int ntypes, const int32_t *T,
                        const uint8_t *Mk, int32_t *use)
{
    launch(c, "dats_select", k_dats_select, dim3((unsigned)((N * K + 255) / 256)), dim3(256), N, K, C, ntypes, T, Mk,
           use, c->flags);
}


// ---- batched replicas: one launch per phase over every replica ----------------
// base[r] .. base[r+1] are replica r's blocks; all replicas share p and precision.

// first pass of the general-lattice replicas (site_lf_body)
template <int P, bool MIXED>
__global__ __launch_bounds__(256) void k_b_site_lf(const RepDev *__restrict__ reps, int R,
                                                   const int64_t *__restrict__ base)
{
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    site_lf_body<P, MIXED>(blockIdx.x - base[r], d.g, d.M, d.psi, d.psi32, d.Bz, d.Tax, d.cell_rng, d.phicoarse,
                           d.phisite);
}

// general-lattice replicas (2x2x2 replicas take k_b_site_s2 in a launch of
// their own, so neither body's registers limit the other's occupancy)
template <int P, bool MIXED>
__global__ __launch_bounds__(256) void k_b_site_gen(const RepDev *__restrict__ reps, int R,
                                                    const int64_t *__restrict__ base)
{
    __shared__ __align__(16) unsigned char smem[general_smem_bytes<MIXED>()];
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    site_general_body<P, MIXED>(blockIdx.x - base[r], d.g, d.M, d.psi, d.psi32, d.Bz, d.Tax, d.qsite, d.qsite32,
                                d.cell_rng, d.site_rank, d.phisite, d.phi_r, d.phicoarse, smem);
}

template <int TC>
__global__ __launch_bounds__(256) void k_b_slot(const RepDev *__restrict__ reps, int R,
                                                const int64_t *__restrict__ base)
{
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    slot_body<TC>(blockIdx.x - base[r], d.g, d.N, (uint32_t)d.K, d.kmul, d.offsets, d.order, d.ijk_r, d.q_r,
                  d.phi_r, d.phisite, d.F, d.Fhop, d.s2, d.dU, d.mask);
}

// nparts blocks per replica: parts part0 .. part0 + nparts - 1
__global__ __launch_bounds__(256) void k_b_move_dU(const RepDev *__restrict__ reps,
                                                   const MoveDev *__restrict__ moves, double *__restrict__ acc,
                                                   int part0, int nparts)
{
    const int r = blockIdx.x / nparts, part = part0 + (int)(blockIdx.x % nparts);
    const MoveDev &mv = moves[r];
    if (!mv.valid) return;
    const RepDev &d = reps[r];
    move_dU_body(part, d.g, d.p, d.M, mv.i, mv.t[0], mv.t[1], mv.t[2], d.psi, d.x, d.y, d.z, d.q, d.cnt, d.slots,
                 d.R, d.H, acc + (int64_t)r * kMoveParts, d.psi_lv);
}

// the moved charge's F row (periodic replicas): w blocks per replica, then K
// one-wave blocks per replica (blocks past a replica's hop count return)
__global__ __launch_bounds__(256) void k_b_frow_w(const RepDev *__restrict__ reps, const MoveDev *__restrict__ moves,
                                                  int nblk)
{
    const int r = blockIdx.x / nblk;
    const MoveDev &mv = moves[r];
    const RepDev &d = reps[r];
    if (!mv.valid || !d.F) return;
    frow_w_body(blockIdx.x % nblk, d.g, d.p, mv.new_site, d.R, d.frow_w);
}

__global__ __launch_bounds__(64) void k_b_frow_b(const RepDev *__restrict__ reps, const MoveDev *__restrict__ moves,
                                                 int Kmax)
{
    const int r = blockIdx.x / Kmax, k = blockIdx.x % Kmax;
    const MoveDev &mv = moves[r];
    const RepDev &d = reps[r];
    if (!mv.valid || !d.F || k >= d.K) return;
    frow_b_body(k, d.g, d.p, mv.rank, mv.new_site, d.K, d.offsets, d.frow_w, d.sigma, d.F);
}

// per-level mode: the coarser levels at every site of every replica.  General
// lattices: one lane per site (blocks only for such replicas); 2x2x2 lattices:
// the orbit kernel, every coarse level of every replica in one launch.
template <int P>
__global__ __launch_bounds__(256) void k_b_coarse(const RepDev *__restrict__ reps, int R,
                                                  const int64_t *__restrict__ base)
{
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    if (!d.phicoarse) return;
    coarse_site_body<P>(d.g, d.psi_lv, (blockIdx.x - base[r]) * (int64_t)blockDim.x + threadIdx.x, d.s2, d.phicoarse);
}

template <int P>
__global__ __launch_bounds__(kCoarseThreads) void k_b_coarse_s2(const RepDev *__restrict__ reps, int R,
                                                     const int64_t *__restrict__ base)
{
    extern __shared__ double sL[];
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    int64_t blk = blockIdx.x - base[r];
    const int level = coarse_s2_level_of(d.g.L, d.g.lstart, blk);
    const int64_t ns = (int64_t)d.g.n * d.g.n * d.g.n;
    coarse_s2_body<P>(d.g, level, d.psi_lv[level], d.phicoarse + (int64_t)(d.g.L - 1 - level) * ns, blk, sL);
}

void launch_b_coarse(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                     int p)
{
    FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_coarse", k_b_coarse<P_>, dim3((unsigned)blocks), dim3(256), 0, reps,
                                     R, base));
}

void launch_b_coarse_s2(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                        int p)
{
    FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_coarse_s2", k_b_coarse_s2<P_>, dim3((unsigned)blocks),
                                     dim3(kCoarseThreads), coarse_s2_shm(p), reps, R, base));
}

int64_t coarse_s2_replica_blocks(int L, int lstart) { return coarse_s2_all_blocks(L, lstart); }

// every replica with 2 x 2 x 2 sites per fine cell: the 8-wave form of that
// body (256 cells per block), as the single-context kernel runs it
template <int P, bool MIXED>
__global__ __launch_bounds__(512) void k_b_site_s2(const RepDev *__restrict__ reps, int R,
                                                   const int64_t *__restrict__ base)
{
    __shared__ __align__(16) unsigned char smem[s2_smem_bytes<MIXED, 8>()];
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    site_s2_body<P, MIXED, 8>(blockIdx.x - base[r], d.g, d.M, d.psi, d.psi32, d.qsite, d.qsite32, d.site_rank, d.Bz,
                              d.Tax, d.phisite, d.phi_r, d.phicoarse, smem);
}

void launch_b_site(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base_s2,
                   int64_t blocks_s2, const int64_t *base_lf, int64_t blocks_lf, const int64_t *base_gen,
                   int64_t blocks_gen, int p, bool mixed)
{
    if (blocks_lf > 0) {
        if (mixed) {
            FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_site", k_b_site_lf<P_, true>, dim3((unsigned)blocks_lf),
                                             dim3(256), 0, reps, R, base_lf));
        } else {
            FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_site", k_b_site_lf<P_, false>, dim3((unsigned)blocks_lf),
                                             dim3(256), 0, reps, R, base_lf));
        }
    }
    if (blocks_s2 > 0) {
        if (mixed) {
            FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_site", k_b_site_s2<P_, true>, dim3((unsigned)blocks_s2),
                                             dim3(512), 0, reps, R, base_s2));
        } else {
            FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_site", k_b_site_s2<P_, false>, dim3((unsigned)blocks_s2),
                                             dim3(512), 0, reps, R, base_s2));
        }
    }
    if (blocks_gen > 0) {
        if (mixed) {
            FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_site", k_b_site_gen<P_, true>, dim3((unsigned)blocks_gen),
                                             dim3(256), 0, reps, R, base_gen));
        } else {
            FMMKMC_DISPATCH_P(p, launch_prof(pr, st, "b_site", k_b_site_gen<P_, false>, dim3((unsigned)blocks_gen),
                                             dim3(256), 0, reps, R, base_gen));
        }
    }
}

void launch_b_slot(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                   int tc)
{
    if (tc == 32)
        launch_prof(pr, st, "b_slot", k_b_slot<32>, dim3((unsigned)blocks), dim3(256), 0, reps, R, base);
    else if (tc == 128)
        launch_prof(pr, st, "b_slot", k_b_slot<128>, dim3((unsigned)blocks), dim3(256), 0, reps, R, base);
    else
        launch_prof(pr, st, "b_slot", k_b_slot<64>, dim3((unsigned)blocks), dim3(256), 0, reps, R, base);
}

void launch_b_move_dU(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const MoveDev *moves, double *acc,
                      int nt, int part0, int nparts, int nlev_max)
{
    const size_t shm = move_dU_shm(nt, nlev_max);
    launch_prof(pr, st, part0 == 0 ? "b_move_dU" : "b_move_dU_side", k_b_move_dU, dim3((unsigned)(R * nparts)),
                dim3(256), shm, reps, moves, acc, part0, nparts);
}

void launch_b_frow(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const MoveDev *moves, int nt, int K)
{
    const int nblk = frow_w_blocks(nt);
    launch_prof(pr, st, "b_frow", k_b_frow_w, dim3((unsigned)(R * nblk)), dim3(256), 0, reps, moves, nblk);
    launch_prof(pr, st, "b_frow", k_b_frow_b, dim3((unsigned)(R * K)), dim3(64), 0, reps, moves, K);
}

}  // namespace fmmkmc
