/*
 * fmmkmc: FMM electrostatics for kinetic Monte Carlo on AMD MI355X (gfx950).
 *
 * Implements the method of Saunders, Grant, Mueller and Thompson, "Fast
 * electrostatic solvers for kinetic Monte Carlo simulations" (arXiv:1905.04065):
 * the energy change dU of every proposed single-charge hop (Sec. 3,
 * Eq. (proposed_energy); periodic boxes Sec. 3.1, Eq. (proposed_energy_sr) plus
 * the far-field terms of Sec. 3.1) and the incremental update of the expansions
 * once a hop is accepted (Sec. 3 "Accept move", Sec. 3.1 "Accept move").
 *
 * Units: Coulomb constant 1, so the energy of charges q_i, q_j at distance r is
 * q_i q_j / r.  Positions are in the box [0, a)^3.
 *
 * Calling conventions (all entry points):
 *   - Return FMMKMC_OK (0) or a positive error code below; on error the
 *     context is unchanged and fmmkmc_last_error() describes the failure.
 *   - Bulk arrays are DEVICE pointers (HIP global memory on the context's
 *     device) unless the parameter says "host".  The caller owns every array it
 *     passes; the library never keeps a pointer to it after the call returns.
 *   - Work is issued on the context's stream.  fmmkmc_propose_lattice() is
 *     asynchronous (synchronise the stream before reading dU); every other
 *     call returns after its results are complete.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef FMMKMC_H
#define FMMKMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fmmkmc_status {
    FMMKMC_OK = 0,
    FMMKMC_EINVAL = 1,      /* bad argument (size, level count, order, index, non-neutral periodic box) */
    FMMKMC_EDOMAIN = 2,     /* a position outside the box (free space) or off the lattice (lattice mode) */
    FMMKMC_ECOINCIDENT = 3, /* two charges at one point, or a target on an occupied point */
    FMMKMC_ECAPACITY = 4,   /* a fine cell holds more charges than cell_capacity */
    FMMKMC_ESTATE = 5,      /* call out of order (e.g. propose before initialise) */
    FMMKMC_EHIP = 6,        /* a HIP runtime call failed */
    FMMKMC_ENOMEM = 7       /* device allocation failed */
};

enum fmmkmc_bc { FMMKMC_FREE = 0, FMMKMC_PERIODIC = 1 };
enum fmmkmc_precision { FMMKMC_FP64 = 0, FMMKMC_MIXED = 1 };

typedef struct fmmkmc_ctx fmmkmc_ctx;

/* Solver parameters (Sec. 5.2: the KMCFMM constructor's levels and terms,
 * Sec. 2.2.1 for the boundary condition). */
typedef struct fmmkmc_params {
    double a;          /* box side, > 0 */
    int bc;            /* FMMKMC_FREE or FMMKMC_PERIODIC (periodic: sum of charges must be 0) */
    int levels;        /* octree levels L, root = level 1, fine level has 8^(L-1) cells;
                          free space L >= 2, periodic L >= 3, L <= 10 */
    int order;         /* expansion order p, 1 <= p <= 16: (p+1)^2 coefficients per expansion */
    int precision;     /* FMMKMC_FP64, or FMMKMC_MIXED: FP32 fine-level local expansions
                          (constant term kept in FP64), FP32 near field and L2P with FP32
                          accumulation; dU subtraction, far field, all accept-step
                          updates and the total energy in FP64 */
    int lattice_n;     /* 0, or n > 0: every charge sits on a site ((i+1/2)h, (j+1/2)h, (k+1/2)h)
                          of the n^3 lattice with h = a/n; enables fmmkmc_propose_lattice() */
    int cell_capacity; /* charge slots per fine cell; 0 picks sites-per-cell (lattice mode)
                          or 4 x the largest initial occupancy (otherwise) */
    int device;        /* HIP device ordinal */
    void *stream;      /* hipStream_t for all work, NULL for the null stream */
    int self_image;    /* periodic boxes: how a proposal removes the moving charge's
                          interaction with its own periodic copies.  0: the terms of
                          Sec. 3.1 (V_box self sum, the constant (6 + 8/sqrt3 +
                          12/sqrt2)/a and 1/2 dE.R'dK); 1: their exact value
                          q^2 (G_self - G(r' - r)), G the conducting-boundary periodic
                          pair potential (Ewald sum): results move at truncation level,
                          and lattice proposals need no per-charge hop table.
                          Ignored in free space. */
    int per_level;     /* 0: fine-level local expansions accumulated over the levels
                          (Alg. "fmm"), every fine cell updated at an accept (Sec. 3
                          "Accept move"); 1: each level keeps only its own
                          interaction-list terms, a proposal sums the levels, and an
                          accept updates per level only the cells whose interaction
                          list holds the moved charge (at most 189 per level and copy
                          instead of every fine cell; the O(log N) accept the
                          Introduction and Sec. 7 point to).  Same result before any
                          accept; after accepts the two differ at truncation level. */
} fmmkmc_params;

/* Create a context for n charges (KMCFMM(positions, charges, r, l), Sec. 5.2).
 * xyz: n x 3 positions, q: n charges; both HOST arrays, copied.
 * Errors: EINVAL, EDOMAIN, ECOINCIDENT, ECAPACITY, EHIP, ENOMEM. */
int fmmkmc_create(const fmmkmc_params *prm, int64_t n, const double *xyz, const double *q,
                  fmmkmc_ctx **out);

/* Build the octree expansions (Alg. "fmm", App. A; periodic: wrapped
 * interaction lists and the lattice-sum far field of Sec. 3.1 with the dipole
 * correction of Sec. 2.2.2 / App. B) and return the total energy (Alg.
 * "fmm_evaluation" plus the far-field energy) in *U_out (host).  Must precede
 * every propose / accept call. */
int fmmkmc_initialise(fmmkmc_ctx *c, double *U_out);

/* propose(P), Sec. 5.2.1: n_groups groups; group g moves charge idx[g] to each
 * of the targets offs[g] .. offs[g+1]-1 (CSR, offs has n_groups+1 entries,
 * offs[0] = 0).  targets: offs[n_groups] x 3, dU: offs[n_groups] outputs.
 * idx, offs, targets, dU are device arrays.  Periodic targets are wrapped into
 * the box.  A slot whose target lies outside the box (free space) gets NaN and
 * the call returns EDOMAIN; a target on an occupied point gets NaN and the call
 * returns ECOINCIDENT (other slots are still valid). */
int fmmkmc_propose(fmmkmc_ctx *c, int64_t n_groups, const int64_t *idx, const int64_t *offs,
                   const double *targets, double *dU);

/* fmmkmc_propose() for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, checks, results and errors, but the per-target work memory is
 * a fixed array inside the library (18 MiB per GPU, held until the process
 * ends; located at the first context creation on that device), so the call
 * allocates nothing.  At most 262144 targets per call (offs[n_groups] larger:
 * EINVAL, nothing computed).  The CSR is checked on the device (EINVAL for
 * offs[0] != 0, decreasing offs or a charge index out of range).  All calls on
 * one GPU share the array: calls that overlap on one GPU (several host threads,
 * or contexts on different streams) race and must be serialised by the caller.
 * Returns after dU is complete. */
int fmmkmc_propose_noalloc(fmmkmc_ctx *c, int64_t n_groups, const int64_t *idx, const int64_t *offs,
                           const double *targets, double *dU);

/* propose_with_dats(C, T, R, M, U), App. C: every charge i has type T[i] in
 * [0, n_types) and may hop to the first C[T[i]] of its K candidate targets
 * R[i][0..K-1] (N x 3K doubles); M[i][k] = 1 allows the hop, 0 forbids it.
 * U[i][k] (N x K) receives dU; forbidden entries and entries with
 * k >= C[T[i]] are "undefined" in the paper and are written as NaN here.
 * C (n_types entries) is a HOST array; T, R, M, U are device arrays. */
int fmmkmc_propose_dats(fmmkmc_ctx *c, int K, const int32_t *C, int n_types, const int32_t *T,
                        const double *R, const uint8_t *M, double *U);

/* Lattice fast path (requires lattice_n > 0): for every charge i and hop k the
 * target is the site at lattice offset offsets[k] (K x 3 HOST ints, |entries| <= 1)
 * from the charge's site, wrapped in periodic boxes.  dU (N x K, device) gets
 * the energy change; slots whose target is occupied or (free space) off the
 * lattice are masked: dU = NaN and mask[i][k] = 0 (mask is an optional N x K
 * device array, valid slots 1).  Asynchronous on the context's stream. */
int fmmkmc_propose_lattice(fmmkmc_ctx *c, int K, const int32_t *offsets, double *dU, uint8_t *mask);

/* accept((i, r')), Sec. 5.2.2: move charge i to new_xyz (HOST, 3 doubles;
 * wrapped in periodic boxes).  dU is recomputed for the move (footnote to
 * Sec. 3.1) and returned in *dU_out (host); then every fine-level local
 * expansion, the multipole expansions of the moved charge's cells on every
 * level, and the far-field coefficients are updated, and U += dU.
 * Errors: EINVAL (bad i), EDOMAIN, ECOINCIDENT (target occupied), ECAPACITY. */
int fmmkmc_accept(fmmkmc_ctx *c, int64_t i, const double new_xyz[3], double *dU_out);

/* Uniform external field E (HOST, 3 doubles; the applied field of Sec. 6.3,
 * here on any box): from the next call on, every proposal and accept adds the
 * work -q E.d done against the field over the hop, d = r' - r (periodic boxes:
 * the minimum-image displacement, i.e. the hop itself for hops shorter than
 * half the box).  The energy reported by fmmkmc_energy() then includes the
 * field's work along the accepted moves (the initial energy does not contain a
 * field term).  Default 0.  Errors: EINVAL (non-finite component). */
int fmmkmc_set_field(fmmkmc_ctx *c, const double E[3]);

/* Current total energy (initial energy plus the accepted dU's), host. */
int fmmkmc_energy(fmmkmc_ctx *c, double *U);

/* Current positions, n x 3 device array. */
int fmmkmc_positions(fmmkmc_ctx *c, double *xyz);

/* Electrostatic potential at m points (device m x 3 array) from every charge
 * except exclude[j] (device, -1 for none): local expansion + near field (+ far
 * field in periodic boxes); out: m device doubles.  Used to check the
 * expansions and the energy. */
int fmmkmc_potential(fmmkmc_ctx *c, int64_t m, const double *xyz, const int64_t *exclude, double *out);

/* Multipole expansion Phi of one cell of the octree (Eq. (multipole_local_expansion),
 * kept current by the accept step's update of the moved charge's cells on every
 * level, Sec. 3 "Accept move").  level in 1..L (root = 1); cell
 * (ix * s + iy) * s + iz with s = 2^(level-1) cells per axis, cell (ix, iy, iz)
 * covering [ix w, (ix+1) w) x ... with w = a / s, expanded about its centre c.
 * out (HOST, (p+1)^2 doubles) gets M_n^m = sum_i q_i conj(R_n^m(r_i - c)) over
 * the charges in the cell, with the regular solid harmonics
 *   R_n^m(x) = (-1)^m |x|^n P_n^m(cos theta) e^{i m phi} / (n+m)!
 * (P_n^m without the Condon-Shortley phase); slot n^2 holds M_n^0, slots
 * n^2 + 2m - 1 and n^2 + 2m hold Re and Im of M_n^m for m = 1..n (the m < 0
 * coefficients are (-1)^m conj(M_n^|m|)).  Level 1 is the whole box, whose
 * multipole the far field uses (Sec. 3.1).  Errors: EINVAL (level or cell out of
 * range), ESTATE (not initialised), EHIP. */
int fmmkmc_multipole(fmmkmc_ctx *c, int level, int64_t cell, double *out);

/* Per-kernel timing: when on, every kernel launch is bracketed by HIP events
 * on the context's stream.  fmmkmc_kernel_time() returns the accumulated time
 * (ms) and launch count of the named kernel since profiling was switched on. */
int fmmkmc_set_profiling(fmmkmc_ctx *c, int on);
int fmmkmc_kernel_time(fmmkmc_ctx *c, const char *name, double *ms, int64_t *launches);

/* Text of the last error on this context (static storage owned by it). */
const char *fmmkmc_last_error(fmmkmc_ctx *c);

/* Free the context and all its device memory. */
int fmmkmc_destroy(fmmkmc_ctx *c);

/* ---- batched replicas --------------------------------------------------
 * Independent KMC systems of uneven sizes run side by side (ensembles, which
 * Sec. 6.4 runs as simultaneous instances) and advance together: each KMC step of Alg. 1 (every proposal's dU, selection of one
 * move, accept) is one launch per phase over all replicas, and the whole step
 * is captured once as a HIP graph and replayed. */
typedef struct fmmkmc_batch fmmkmc_batch;

/* Group n initialised lattice-mode contexts (HOST array ctx[n]) that share
 * expansion order, precision and device; the contexts stay owned by the
 * caller and must outlive the batch.  Every replica proposes the same K hops
 * offsets[k] (K x 3 HOST ints, |entries| <= 1, as in fmmkmc_propose_lattice).
 * stream: hipStream_t for the batch's work, not the legacy null stream (a step
 * is captured as a graph on it); NULL: the batch creates a stream of its own.
 * Errors: EINVAL (n < 1, mixed orders/precisions/devices, no lattice, bad K),
 * ESTATE (a context not initialised), EHIP, ENOMEM. */
int fmmkmc_batch_create(int n, fmmkmc_ctx *const *ctx, int K, const int32_t *offsets, void *stream,
                        fmmkmc_batch **out);

/* Propensities of the selection (Alg. 1, r = r(dU) per proposed hop):
 *   kind 0 (the default): 1 for every valid slot, a choice that does not look
 *          at dU (one uniform per replica and step, no time increment);
 *   kind 1: nu exp(-beta dU), the Boltzmann factor of the full KMC runs (Sec. 6);
 *   kind 2: nu min(1, exp(-beta dU)), the Metropolis form.
 * Kinds 1 and 2 take two uniforms per replica and step and return Delta t.
 * The exponent -beta dU is capped at 600 (rates stay finite when summed).
 * Errors: EINVAL (kind not 0..2; for kinds 1, 2: nu <= 0, beta < 0 or either
 * not finite), EHIP.  The step graph is captured again at the next step. */
int fmmkmc_batch_set_rates(fmmkmc_batch *b, int kind, double nu, double beta);

/* n_steps KMC steps on every replica r (Alg. 1).  Step s: dU of every
 * (charge, hop) slot; the propensities r_j of the slots j = i * K + k in slot
 * order (masked slots: 0), cumulative sums R_j and total Q; the move taken is
 * the slot with R_{j-1} < T <= R_j, where
 *   kind 0: T = floor(u V) + 1, V = Q the number of valid slots, i.e. valid
 *           slot number floor(u V); u = u[s n + r];
 *   kinds 1, 2: T = Q zeta with zeta = 1 - u[2 (s n + r)], and the time
 *           increment Delta t = -log(xi) / Q with xi = 1 - u[2 (s n + r) + 1];
 * u: DEVICE doubles, uniform in [0, 1), n_steps x n (kind 0) or n_steps x n x 2.
 * Then that move is accepted (dU recomputed from the FP64 expansions, every
 * expansion updated, U += dU).  A replica with Q = 0 does not move.  Outputs
 * (DEVICE arrays of n_steps x n, each may be NULL): moved[s n + r] the charge
 * moved (-1 if none), site[s n + r] its new lattice site (lattice order),
 * dU[s n + r] the accepted dU (NaN if none), dt[s n + r] Delta t (kinds 1, 2;
 * +inf if Q = 0; NaN for kind 0).  Returns after the steps are complete; the
 * contexts' energies are updated and their single-context calls see the new
 * configuration. */
int fmmkmc_batch_step(fmmkmc_batch *b, int n_steps, const double *u, int64_t *moved, int64_t *site, double *dU,
                      double *dt);

/* Copy replica r's dU and mask of the last proposal pass (N_r x K device arrays;
 * mask may be NULL). */
int fmmkmc_batch_proposals(fmmkmc_batch *b, int r, double *dU, uint8_t *mask);

/* Autotuner: time the tile choices of the phases that have them (charges per
 * block of the slot gather, threads per block of the sweep) on this batch and
 * keep the fastest; the step graph is captured again with them.  rounds: timed
 * launches per candidate (>= 1).  The choices can be read with
 * fmmkmc_batch_info(). */
int fmmkmc_batch_tune(fmmkmc_batch *b, int rounds);

/* Slots per step (sum of N_r K) and the current tile choices. */
int fmmkmc_batch_info(fmmkmc_batch *b, int64_t *slots_per_step, int *slot_tile, int *sweep_block);

/* Per-phase timing of batched steps: with profiling on, steps run as plain
 * launches (not the graph) bracketed by HIP events; names as in the kernels
 * ("b_site", "b_slot", "b_select", "b_sweep", ...). */
int fmmkmc_batch_set_profiling(fmmkmc_batch *b, int on);
int fmmkmc_batch_kernel_time(fmmkmc_batch *b, const char *name, double *ms, int64_t *launches);

/* Text of the last error on this batch. */
const char *fmmkmc_batch_last_error(fmmkmc_batch *b);

/* Free the batch (not its contexts). */
int fmmkmc_batch_destroy(fmmkmc_batch *b);

/* ---- slab between grounded plates ---------------------------------------
 * Dirichlet boundaries of Sec. 2.2.2: the potential is zero on the planes
 * z = 0 and z = a/2 (the plates); x and y are periodic with period a; a
 * uniform external field E_z along z (Sec. 6.3: an applied potential
 * difference) adds -E_z q z to the energy of each charge.  As in the paper, the
 * slab is extended by its first mirror image (charge -q at (x, y, a - z)) and
 * the doubled system is treated with the periodic algorithm (conducting
 * boundary), whose potential vanishes on both planes by symmetry.  Energies are
 * those of the physical charges: half the periodic energy of the doubled
 * system plus the field term.  A hop moves a charge and its mirror together;
 * its dU is (dU_i + dU_m + X) / 2 - E_z q dz, with dU_i and dU_m the periodic
 * single-move values (each with the partner at its old place) and X the pair
 * correction q_i q_m [G(r_i'-r_m') - G(r_i'-r_m) - G(r_i-r_m') + G(r_i-r_m)],
 * G the periodic pair potential, tabulated per (site height, hop) with an Ewald
 * sum.  Lattice proposals only; slabs do not join batches. */
typedef struct fmmkmc_slab fmmkmc_slab;

/* prm as for fmmkmc_create (bc is ignored: the doubled system is periodic;
 * lattice_n must be even and > 0, levels >= 3); n physical charges at HOST
 * positions xyz (n x 3, lattice sites with 0 <= z < a/2) with HOST charges q
 * (any total charge); ez: the field E_z.  Errors: EINVAL, EDOMAIN (a charge
 * outside 0 <= z < a/2), and those of fmmkmc_create. */
int fmmkmc_slab_create(const fmmkmc_params *prm, int64_t n, const double *xyz, const double *q, double ez,
                       fmmkmc_slab **out);

/* Build the expansions of the doubled system; *U_out (host, may be NULL) gets
 * the energy of the physical charges. */
int fmmkmc_slab_initialise(fmmkmc_slab *s, double *U_out);

/* dU of every hop of every physical charge, as fmmkmc_propose_lattice (K x 3
 * HOST offsets in -1..1, DEVICE dU and mask of n x K).  The hop set must be
 * closed under (dx, dy, dz) -> (dx, dy, -dz).  A hop is masked (NaN, mask 0)
 * when its target is occupied or lies outside 0 <= z < a/2 (hops do not wrap
 * in z); x and y wrap.  Errors: EINVAL, ESTATE, EHIP. */
int fmmkmc_slab_propose_lattice(fmmkmc_slab *s, int K, const int32_t *offsets, double *dU, uint8_t *mask);

/* Move physical charge i to new_xyz (host, a free lattice site with
 * 0 <= z < a/2) together with its mirror; *dU_out (host) gets the dU of the
 * move, recomputed on the FP64 path.  Errors: as fmmkmc_accept, EDOMAIN for a
 * target outside the slab; if the mirror's move fails after the charge moved,
 * the slab must be initialised again (ESTATE until then). */
int fmmkmc_slab_accept(fmmkmc_slab *s, int64_t i, const double new_xyz[3], double *dU_out);

/* Energy of the physical charges (host). */
int fmmkmc_slab_energy(fmmkmc_slab *s, double *U);

/* Positions of the physical charges (n x 3 DEVICE array). */
int fmmkmc_slab_positions(fmmkmc_slab *s, double *xyz);

/* Text of the last error on this slab (NULL: of the last failed create). */
const char *fmmkmc_slab_last_error(fmmkmc_slab *s);

/* Free the slab and its doubled system. */
int fmmkmc_slab_destroy(fmmkmc_slab *s);

#ifdef __cplusplus
}
#endif

#endif
