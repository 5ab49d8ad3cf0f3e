// Replica descriptors for the batched kernels: many independent lattice
// systems (KMC replicas of uneven sizes) advanced by one launch per phase.
// Each replica is an ordinary context; RepDev is a device-resident view of its
// arrays, and a batched kernel maps each block to (replica, local block)
// through a prefix table of per-replica block counts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace fmmkmc {

struct RepDev {
    Geo g;
    int64_t M, N;
    int L, p, nt, K, s2, cap;
    uint32_t kmul;  // floor(2^32 / K)
    // fine-level local expansions (coefficient-major) and the level pointers of the multipoles
    double *psi;
    float *psi32;
    double *const *phi_lv;
    double *const *psi_lv;  // local expansions of every level (per-level mode)
    double *phicoarse;      // per-level mode: the coarse levels' potential at each site
    // charges
    double *x, *y, *z, *q;
    int32_t *cell, *slot, *site, *cnt, *slots, *rank_of;
    // site tables (site order)
    int32_t *site_charge, *site_rank;
    double *qsite;
    float *qsite32;
    int32_t *cell_rng;
    double *phisite;
    // by rank
    int32_t *order, *ijk_r;
    double *q_r, *phi_r, *F;
    double *Fhop;  // exact self-image option: per-hop table instead of F
    double *frow_w;  // the F row of a moved charge: R K1 at its new site (nt)
    // hops and the proposal output of this replica ([charge][hop])
    int32_t *offsets;
    double *dU;
    uint8_t *mask;
    // far field
    double *R, *GR, *Kf, *H, *C, *A, *Bz, *Tax, *sigma;
    int32_t *cz;
    int ncz;
};

// the move a replica makes in the current step (written by the selection kernel)
struct MoveDev {
    int valid;         // 0: no valid slot, the replica does not move
    int64_t i;         // charge
    int64_t slot;      // selected slot i * K + k
    int64_t new_site;  // lattice order
    int32_t rank;
    double t[3];       // new position
    Move mv;
    Book bk;
};

// replica owning block b of a batched launch: base[r] <= b < base[r + 1]
__device__ inline int find_rep(const int64_t *__restrict__ base, int R, int64_t b)
{
    int lo = 0, hi = R;  // invariant: base[lo] <= b < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// launchers of the batched kernels (grids: one block range per replica)
// site potentials: replicas with 2 x 2 x 2 sites per fine cell (256 cells per
// 512-thread block), then the two passes of the general-lattice replicas (the
// local expansion, far field and coarse levels per site; the near field), one
// launch each (a replica has blocks in the s2 table or in the other two)
void launch_b_site(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base_s2,
                   int64_t blocks_s2, const int64_t *base_lf, int64_t blocks_lf, const int64_t *base_gen,
                   int64_t blocks_gen, int p, bool mixed);
void launch_b_slot(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                   int tc);
// parts [part0, part0 + nparts) of every replica's move dU
// nlev_max: the most levels any replica evaluates in the dU of its move (1, or
// L - 1 in per-level mode)
void launch_b_move_dU(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const MoveDev *moves, double *acc,
                      int nt, int part0, int nparts, int nlev_max);
void launch_b_frow(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const MoveDev *moves, int nt, int K);
void launch_b_sweep(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                    int p, const MoveDev *moves, int block);
void launch_b_path(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                   const MoveDev *moves);
// per-level mode: the commit on every level of every replica (instead of the sweep)
void launch_b_levels(Profiler &pr, hipStream_t st, const RepDev *reps, int R, int p, const MoveDev *moves, int Lmax,
                     int lstart);
// per-level mode: the coarse levels' potential at every site of every replica
void launch_b_coarse(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                     int p);
// ... on 2x2x2 lattices, the orbit kernel for every coarse level of every replica (one launch)
void launch_b_coarse_s2(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base, int64_t blocks,
                        int p);
// blocks of that kernel for one 2x2x2 replica with L levels, coarse levels lstart .. L-1
int64_t coarse_s2_replica_blocks(int L, int lstart);
void launch_b_book(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const MoveDev *moves);
void launch_b_far(Profiler &pr, hipStream_t st, const RepDev *reps, int R, const int64_t *base_far,
                  int64_t blocks_far, const int64_t *base_a, int64_t blocks_a, const int64_t *base_b,
                  int64_t blocks_b, const MoveDev *moves);

}  // namespace fmmkmc

// host mirrors of a context after batched steps (api.hip)
void refresh_mirrors(fmmkmc_ctx *c);
