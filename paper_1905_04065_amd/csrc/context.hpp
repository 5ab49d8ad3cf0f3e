// Library context: device state of one FMM-KMC system and host mirrors of the
// bookkeeping needed to validate an accepted move without a device round trip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/fmmkmc.h"

namespace fmmkmc {

constexpr int kMaxOrder = 16;
constexpr int kMaxLevels = 10;
constexpr int kMaxHops = 64;       // hop offsets per lattice proposal call
constexpr int kMaxLattice = 1024;  // lattice sites per axis (10-bit packed coordinates)

// geometry passed by value to kernels
struct Geo {
    double a;      // box side
    double w;      // fine cell width
    double h;      // lattice spacing (lattice mode), else 0
    int nc;        // fine cells per axis, 2^(L-1)
    int n;         // lattice sites per axis (lattice mode), else 0
    int periodic;  // 1 periodic, 0 free space
    int cap;       // slots per fine cell
    int tab_ok;    // lattice: every squared site offset of a near field is below kInvTab
    int self_exact;  // periodic: proposals take the exact self-image change (Ewald), not the
                     // V_box self sum + constant + 1/2 dE.R'dK
    int per_level;   // local expansions kept per level (no L2L); evaluation sums the levels
    int L;           // levels (root = 1): the fine level
    int lstart;      // first level with an interaction list (periodic 2, free space 3)
    int q32;         // lattice: an FP32 copy of the site charges exists (mixed precision, or every
                     // charge is exactly an FP32 number)
    int ncoarse;     // per-level mode, lattice: per-site arrays of the coarse levels' potential (0: none;
                     // 2x2x2 lattices one per level, array a holding level L-1-a; other lattices one
                     // array of all levels)
    double field[3];  // uniform external field E: a hop by d adds -q E.d
};

// displacement of a hop from r to t: t - r, in periodic boxes its minimum image
__host__ __device__ inline double hop_component(const Geo &g, double d)
{
    return g.periodic ? d - g.a * floor(d / g.a + 0.5) : d;
}

// -E.d of a hop from r to t (times q: the field's share of its dU)
__host__ __device__ inline double field_work(const Geo &g, double dx, double dy, double dz)
{
    return -(g.field[0] * hop_component(g, dx) + g.field[1] * hop_component(g, dy) + g.field[2] * hop_component(g, dz));
}

// entries of the 1/sqrt(k) table of the lattice near field (integer squared offsets)
constexpr int kInvTab = 512;

struct Profiler {
    bool on = false;
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::map<std::string, std::pair<double, int64_t>> total;  // ms, launches
    void resolve();
};

struct FarField {
    double *K = nullptr;      // multipole of the box about its centre (nt)
    double *H = nullptr;      // local expansion of the copies in V_inf (nt)
    double *R = nullptr;      // far operator, [k][n] (nt x nt)
    double *GR = nullptr;     // Chebyshev map times R, nonzero rows only, column-major [nt][ncz]
    int32_t *cz = nullptr;    // index in the (p+1)^3 coefficient array of each nonzero row
    int ncz = 0;
    double *C = nullptr;      // Chebyshev coefficients (p+1)^3
    double *A = nullptr;      // lattice: [n][p+1][p+1] partial sums over x
    double *Bz = nullptr;     // lattice: [n][n][p+1] partial sums over x and y
    double *Tax = nullptr;    // lattice: T_c(xi) at the n lattice coordinates [n][p+1]
    double *sigma = nullptr;  // lattice: V_inf self-energy factor per site [n^3]
};

}  // namespace fmmkmc

struct fmmkmc_ctx {
    // parameters
    double a = 0, h = 0;
    int bc = 0, L = 0, p = 0, nt = 0, prec = 0, lat_n = 0, cap = 0, device = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;        // library-owned side stream (accept: F row beside the sweep)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t N = 0;
    int nc = 0;
    int64_t M = 0;        // fine cells
    bool s2 = false;      // lattice with 2x2x2 sites per fine cell
    bool initialised = false;
    bool dev_ahead = false;  // batched steps moved charges: host mirrors are stale
    int near_tab_ok = 0;     // lattice: see Geo::tab_ok
    double U = 0;
    double field[3] = {0.0, 0.0, 0.0};  // uniform external field (fmmkmc_set_field)
    std::string err;
    fmmkmc::Profiler prof;

    // charges (device)
    double *x = nullptr, *y = nullptr, *z = nullptr, *q = nullptr;
    int32_t *cell = nullptr, *slot = nullptr, *site = nullptr;
    int32_t *cell_cnt = nullptr, *cell_slots = nullptr;
    int32_t *site_charge = nullptr;  // lattice: charge on each site or -1, in site order
                                     // (cell-major on the 2x2x2 path, lattice order otherwise)
    // lattice: charges ranked in site order (spatial locality of the per-slot
    // gathers); by rank: charge index, charge, packed site coordinates
    // (i<<20 | j<<10 | k); the hop table F is stored by rank as well
    int32_t *order = nullptr;
    int32_t *rank_of = nullptr;      // lattice: rank of each charge (device copy of hrank)
    double *q_r = nullptr;
    int32_t *ijk_r = nullptr;
    double *qsite = nullptr;         // lattice: charge per site (0 if vacant), site order
    float *qsite32 = nullptr;
    int32_t *cell_rng = nullptr;     // lattice: [nc][2] first and last site index of each fine cell, per axis

    // expansions (device), coefficient-major [k][cells]
    std::vector<double *> phi_lv, psi_lv;  // index = level 1..L
    double **d_phi_ptrs = nullptr;         // device copy of phi_lv
    double **d_psi_ptrs = nullptr;         // device copy of psi_lv
    int per_level = 0;                     // levels kept apart (see fmmkmc_params)
    double *phicoarse = nullptr;           // per-level, lattice: the levels above the fine one at each site
    float *psi32 = nullptr;                // mixed: FP32 copy of psi_lv[L]
    double *phisite = nullptr;             // lattice: potential per vacant site (NaN if occupied), site order
    double *phi_r = nullptr;               // lattice: phi_occ of each charge, by rank
    int32_t *site_rank = nullptr;          // lattice: rank of the charge on each site or -1, site order

    // operators (device)
    std::vector<double *> m2m;   // [level] 8 matrices [c][n][k] (parent level 1..L-1)
    std::vector<double *> l2l;   // [level] 8 matrices [c][n][k] (child level 2..L)
    double *m2l = nullptr;       // 316 unit-width matrices [o][n][k]
    int32_t *m2l_index = nullptr;  // 343 entries: (dx+3)*49 + (dy+3)*7 + (dz+3) -> o or -1
    double *scale = nullptr;     // [level][2][nt]: w^-deg(n) and w^-(deg(k)+1)
    fmmkmc::FarField far;

    // lattice proposal table (periodic): F[i][k] per charge and hop; with the
    // exact self-image option a per-hop table Fhop[k] instead
    int self_exact = 0;
    double *F = nullptr;
    double *Fhop = nullptr;
    double *frow_w = nullptr;         // F row of a moved charge: R K1 at its new site (nt)
    std::vector<int32_t> F_offsets;   // 3K ints the table was built for
    int32_t *d_offsets = nullptr;     // device copy of the current hop offsets
    int d_offsets_K = 0;

    // scratch
    double *scr = nullptr;
    size_t scr_bytes = 0;
    int32_t *flags = nullptr;   // device error flags
    int64_t *iota = nullptr;    // 0..N-1
    double *acc_buf = nullptr;  // accept: target, charge index, dU (32 doubles)
    double *red = nullptr;      // reduction partials

    // host mirrors
    std::vector<double> hx, hy, hz, hq;
    std::vector<int32_t> hcell, hslot, hsite, hcnt, hslots, hsite_charge, hrank;
};
