// Kernel launchers shared by the C-ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "context.hpp"
#include "device.hpp"

namespace fmmkmc {

// Launch on stream s; with profiling on, bracket with HIP events on that stream.
template <typename Kern, typename... Args>
inline void launch_prof(Profiler &pr, hipStream_t s, const char *name, Kern k, dim3 grid, dim3 block, size_t shm,
                        Args... args)
{
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return;
    hipEvent_t a = nullptr, b = nullptr;
    if (pr.on) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
    }
    hipLaunchKernelGGL(k, grid, block, shm, s, args...);
    if (pr.on) {
        (void)hipEventRecord(b, s);
        pr.pending.push_back({name, a, b});
    }
}

template <typename Kern, typename... Args>
inline void launch_on(fmmkmc_ctx *c, hipStream_t s, const char *name, Kern k, dim3 grid, dim3 block, size_t shm,
                      Args... args)
{
    launch_prof(c->prof, s, name, k, grid, block, shm, args...);
}

// Launch on the context's stream.
template <typename Kern, typename... Args>
inline void launch_shm(fmmkmc_ctx *c, const char *name, Kern k, dim3 grid, dim3 block, size_t shm, Args... args)
{
    launch_on(c, c->stream, name, k, grid, block, shm, args...);
}

template <typename Kern, typename... Args>
inline void launch(fmmkmc_ctx *c, const char *name, Kern k, dim3 grid, dim3 block, Args... args)
{
    launch_shm(c, name, k, grid, block, 0, args...);
}

// an accepted move as the commit kernels see it
struct Move {
    double ox, oy, oz;   // old position (in the box)
    double nx, ny, nz;   // new position (in the box)
    double q;
    int ogx, ogy, ogz;   // fine-cell coordinates of the old position
    int ngx, ngy, ngz;   // and of the new one
};

// bookkeeping of an accepted move: positions, cell slots, site tables
struct Book {
    int64_t i;
    double nx, ny, nz, q;
    int64_t old_cell, new_cell;
    int old_slot, new_slot;
    int moved_j;          // charge moved into old_slot (-1 if none)
    int old_cnt, new_cnt; // counts after the move
    int64_t new_site;     // lattice order, -1 without a lattice
    int64_t old_sord, new_sord;  // site order (cell-major on the 2x2x2 path)
    int32_t new_ijk;
    int32_t rank;
    int s2;               // lattice with 2x2x2 sites per fine cell (cell-major site order)
    int same_cell;        // the move stays inside one fine cell: slots unchanged
};

struct CommitArgs {
    int64_t i;
    double old_pos[3], new_pos[3], q;
    int old_g[3], new_g[3];
    int64_t old_cell, new_cell;
    int old_slot, new_slot, moved_j, old_cnt, new_cnt;
    int64_t old_site, new_site;  // lattice order, -1 without a lattice
    int64_t old_sord, new_sord;  // the same sites in the device's site order
    int32_t new_ijk;             // packed coordinates of the new site
    int32_t rank = 0;            // the moved charge's rank in site order
};

Geo make_geo(const fmmkmc_ctx *c);

// setup
void launch_p2m(fmmkmc_ctx *c, const Geo &g);
void launch_upward(fmmkmc_ctx *c);
void launch_downward(fmmkmc_ctx *c);
void launch_far_refresh(fmmkmc_ctx *c, hipStream_t st = nullptr);  // st: nullptr = the context stream
void launch_shadow(fmmkmc_ctx *c);
// propose
void launch_point_phi(fmmkmc_ctx *c, const Geo &g, int64_t m, const double *xyz, const int64_t *pidx,
                      const int64_t *exclude, int with_far, double *out, const char *name,
                      bool fp64 = false);
void launch_site_phi(fmmkmc_ctx *c, const Geo &g);
// per-level mode, lattice: the levels above the fine one at every site (phicoarse)
void launch_coarse_sites(fmmkmc_ctx *c, const Geo &g);
void launch_slot_lattice(fmmkmc_ctx *c, const Geo &g, int K, double *dU, uint8_t *mask);
// exact self-image option: Fhop[k] = G_self - G(h offsets[k]) for the K hops
void launch_self_hops(fmmkmc_ctx *c, int K);
// blocks of the general-geometry site kernel for an n^3 lattice
int64_t general_site_blocks(int n, int nc);
void launch_sigma(fmmkmc_ctx *c, const Geo &g);
// F rows of the charges of ranks first..first+count-1
void launch_f_rows(fmmkmc_ctx *c, const Geo &g, int64_t count, int K, int64_t first);
// work: at least 8 S doubles; use: optional per-slot flag (0 = skip, NaN out)
void launch_generic(fmmkmc_ctx *c, const Geo &g, int64_t S, const double *tgt, const int64_t *charge, double *dU,
                    double *work, const int32_t *use = nullptr);
void launch_div_index(fmmkmc_ctx *c, int64_t S, int K, int64_t *charge);
void launch_expand_groups(fmmkmc_ctx *c, int64_t G, const int64_t *idx, const int64_t *offs, int64_t *charge);
void launch_dats_select(fmmkmc_ctx *c, int64_t N, int K, const int32_t *C, int ntypes, const int32_t *T,
                        const uint8_t *Mk, int32_t *use);
// accept
// dU of a move as kMoveParts partial sums out[0..kMoveParts-1] (added by the
// caller in index order): part 0 reads the fine-level expansions (so it must
// precede the sweep), parts 1..3 the cell lists and the far-field tables (so
// they must precede the bookkeeping and the far-field update).  Launches
// parts [part0, part0 + nparts) on stream st (the context's stream if null).
constexpr int kMoveParts = 4;
void launch_move_dU(fmmkmc_ctx *c, const Geo &g, int64_t i, const double t[3], double *out,
                    hipStream_t st = nullptr, int part0 = 0, int nparts = kMoveParts);
// F row of one charge (rank, its new lattice site s) on stream st
void launch_f_row1(fmmkmc_ctx *c, const Geo &g, int K, int64_t rank, int64_t s, hipStream_t st);
// sweep on the context stream; path and bookkeeping on side (they touch neither
// the fine-level expansions nor anything the sweep reads)
void launch_commit(fmmkmc_ctx *c, const Geo &g, const CommitArgs &a, hipStream_t side);

}  // namespace fmmkmc
