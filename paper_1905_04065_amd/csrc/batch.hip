// Batched replicas: many independent lattice systems advanced by one launch
// per phase of a KMC step (Alg. 1: every proposal's dU, selection of one move,
// accept), the whole step captured once as a HIP graph.
//
// Phases of a step, each one launch over every replica (block ranges per
// replica, see batch.hpp); b_frow, b_path, b_book and the far field run on a
// side stream beside b_sweep:
//   b_site, b_slot      the proposal pass (Sec. 3: dU of every hop)
//   b_count, b_select   the move (Alg. 1): slot j with R_{j-1} < T <= R_j over
//                       the cumulative propensities in slot order, then the
//                       accept arguments built on the device
//   b_move_dU           dU of the move recomputed (footnote to Sec. 3.1)
//   b_frow              the moved charge's row of the hop table
//   b_sweep, b_path     every fine-level local expansion, the multipole path
//   b_book              positions, cell slots, site tables
//   b_far_refresh, b_cheb_a, b_cheb_b   far field (Sec. 3.1)
//   b_finish            U += dU, outputs, step counter
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fmmkmc.h"
#include "batch.hpp"
#include "hostutil.hpp"
#include "kernels.hpp"

using namespace fmmkmc;

namespace {

constexpr int kSelLane = 32;                // consecutive slots per lane
constexpr int kSelChunk = 256 * kSelLane;  // slots per counting block

// Propensity of a valid slot (Alg. 1: r = r(dU)); masked slots have none.
//   kind 0: 1 (a uniform choice among the valid slots, which does not look at dU)
//   kind 1: nu exp(-beta dU), the Boltzmann factor the full KMC runs of Sec. 6 use
//   kind 2: nu min(1, exp(-beta dU)), the Metropolis form
// The exponent is capped at 600 so that a sum over any realistic number of
// slots stays finite.
struct Rates {
    int kind;
    double nu, beta;
};

__device__ inline double slot_rate(const Rates &rt, uint8_t valid, double dU)
{
    if (!valid) return 0.0;
    if (rt.kind == 0) return 1.0;
    const double x = -rt.beta * dU;
    if (rt.kind == 2) return x >= 0.0 ? rt.nu : rt.nu * exp(x);
    return rt.nu * exp(x < 600.0 ? x : 600.0);
}

// Propensities of the kSelLane slots b0, b0 + 1, ... of a replica (0 past its
// end).  Kind 0 reads only the mask; whole runs use vector loads (the batch's
// own dU and mask arrays, 256-byte aligned, and b0 a multiple of kSelLane).
__device__ inline void lane_rates(const RepDev &d, const Rates &rt, int64_t b0, double (&w)[kSelLane])
{
    const int64_t S = d.N * d.K;
    uint8_t v[kSelLane];
    double u[kSelLane];
    if (b0 + kSelLane <= S) {
        const uint4 *m4 = (const uint4 *)(d.mask + b0);
#pragma unroll
        for (int h = 0; h < kSelLane / 16; ++h) {
            const uint4 x = m4[h];
            const uint32_t wd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) v[16 * h + k] = (uint8_t)(wd[k >> 2] >> (8 * (k & 3)));
        }
        if (rt.kind != 0) {
            const double2 *u2 = (const double2 *)(d.dU + b0);
#pragma unroll
            for (int h = 0; h < kSelLane / 2; ++h) {
                const double2 x = u2[h];
                u[2 * h] = x.x;
                u[2 * h + 1] = x.y;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < kSelLane; ++k) {
            const bool in = b0 + k < S;
            v[k] = in ? d.mask[b0 + k] : 0;
            u[k] = (in && rt.kind != 0) ? d.dU[b0 + k] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < kSelLane; ++k) w[k] = slot_rate(rt, v[k], rt.kind != 0 ? u[k] : 0.0);
}

// summed propensity of each chunk of kSelChunk consecutive slots of a replica
// (each lane adds its kSelLane slots in order, then a tree over the lanes)
__global__ __launch_bounds__(256) void k_b_count(const RepDev *__restrict__ reps, int R,
                                                 const int64_t *__restrict__ base, Rates rt,
                                                 double *__restrict__ wsum)
{
    __shared__ double red[256];
    const int r = find_rep(base, R, blockIdx.x);
    const RepDev &d = reps[r];
    const int64_t b0 = (blockIdx.x - base[r]) * (int64_t)kSelChunk + (int64_t)threadIdx.x * kSelLane;
    double w[kSelLane];
    lane_rates(d, rt, b0, w);
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < kSelLane; ++k) c += w[k];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsum[blockIdx.x] = red[0];
}

// prefix sums over the 256 lanes of a block: lane t covers (*lo, *hi] with
// *lo the inclusive sum of lane t - 1 (0 for lane 0), so the lanes' intervals
// tile (0, *total] exactly
__device__ void block_scan(double v, double *sm, double *lo, double *hi, double *total)
{
    const int t = threadIdx.x;
    sm[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const double x = t >= off ? sm[t - off] : 0.0;
        __syncthreads();
        sm[t] += x;
        __syncthreads();
    }
    *hi = sm[t];
    *lo = t > 0 ? sm[t - 1] : 0.0;
    *total = sm[255];
    __syncthreads();
}

// the accept arguments of moving charge i by hop k (the device-side
// counterpart of what fmmkmc_accept derives on the host)
__device__ void prepare_move(const RepDev &d, int64_t slot, MoveDev &m)
{
    const int K = d.K, n = d.g.n, nc = d.g.nc, cap = d.cap;
    const int64_t i = slot / K;
    const int k = (int)(slot - i * K);
    const int32_t os = d.site[i];
    const int si = os / (n * n), sj = (os / n) % n, sk = os % n;
    int ti = si + d.offsets[3 * k], tj = sj + d.offsets[3 * k + 1], tk = sk + d.offsets[3 * k + 2];
    if (d.g.periodic) {
        ti = posmod(ti, n);
        tj = posmod(tj, n);
        tk = posmod(tk, n);
    }
    const int64_t ns = ((int64_t)ti * n + tj) * n + tk;
    const double h = d.g.h, w = d.g.w;
    const double nx = (ti + 0.5) * h, ny = (tj + 0.5) * h, nz = (tk + 0.5) * h;
    const double ox = d.x[i], oy = d.y[i], oz = d.z[i], q = d.q[i];
    const int ogx = fine_coord(ox, w, nc), ogy = fine_coord(oy, w, nc), ogz = fine_coord(oz, w, nc);
    const int ngx = fine_coord(nx, w, nc), ngy = fine_coord(ny, w, nc), ngz = fine_coord(nz, w, nc);
    const int64_t old_cell = d.cell[i], new_cell = cell_id(nc, ngx, ngy, ngz);
    const int old_slot = d.slot[i];
    int moved_j = -1, old_cnt = d.cnt[old_cell], new_slot = old_slot, new_cnt = d.cnt[new_cell];
    if (new_cell != old_cell) {
        const int last = d.cnt[old_cell] - 1;
        const int jlast = d.slots[old_cell * cap + last];
        moved_j = jlast != i ? jlast : -1;
        old_cnt = last;
        new_slot = d.cnt[new_cell];
        new_cnt = d.cnt[new_cell] + 1;
    }
    m.valid = 1;
    m.i = i;
    m.slot = slot;
    m.new_site = ns;
    m.rank = d.rank_of[i];
    m.t[0] = nx;
    m.t[1] = ny;
    m.t[2] = nz;
    Move &mv = m.mv;
    mv.ox = ox;
    mv.oy = oy;
    mv.oz = oz;
    mv.nx = nx;
    mv.ny = ny;
    mv.nz = nz;
    mv.q = q;
    mv.ogx = ogx;
    mv.ogy = ogy;
    mv.ogz = ogz;
    mv.ngx = ngx;
    mv.ngy = ngy;
    mv.ngz = ngz;
    Book &b = m.bk;
    b.i = i;
    b.nx = nx;
    b.ny = ny;
    b.nz = nz;
    b.q = q;
    b.old_cell = old_cell;
    b.new_cell = new_cell;
    b.old_slot = old_slot;
    b.new_slot = new_slot;
    b.moved_j = moved_j;
    b.old_cnt = old_cnt;
    b.new_cnt = new_cnt;
    b.new_site = ns;
    b.old_sord = d.s2 ? s2_site(nc, si, sj, sk) : (int64_t)os;
    b.new_sord = d.s2 ? s2_site(nc, ti, tj, tk) : ns;
    b.new_ijk = (ti << 20) | (tj << 10) | tk;
    b.rank = m.rank;
    b.s2 = d.s2;
    b.same_cell = old_cell == new_cell ? 1 : 0;
}

// One block per replica: the first slot j (slot order i * K + k) whose
// cumulative propensity R_j reaches the target T, R_{j-1} < T <= R_j (Alg. 1):
//   kind 0: T = floor(u V) + 1 with V valid slots (the valid slot number floor(u V));
//   kinds 1, 2: T = Q zeta with Q the total propensity and zeta = 1 - u in (0, 1].
// Then the accept arguments of that move.  The chunk sums and the in-chunk
// scan add in different orders, so a target within rounding of a chunk edge
// falls back on the chunk's last slot with a propensity.
__global__ __launch_bounds__(256) void k_b_select(const RepDev *__restrict__ reps, int R,
                                                  const int64_t *__restrict__ cbase,
                                                  const double *__restrict__ wsum, Rates rt,
                                                  const double *__restrict__ u, const int32_t *__restrict__ step,
                                                  MoveDev *__restrict__ moves, double *__restrict__ Qout)
{
    __shared__ double sm[256];
    __shared__ int64_t s_chunk, s_slot;
    __shared__ double s_target;
    const int r = blockIdx.x;
    const RepDev &d = reps[r];
    const int t = threadIdx.x;
    const int64_t c0 = cbase[r], nch = cbase[r + 1] - c0;
    const int64_t per = (nch + 255) / 256;
    const int64_t k0 = (int64_t)t * per < nch ? (int64_t)t * per : nch;
    const int64_t k1 = k0 + per < nch ? k0 + per : nch;
    double mine = 0.0;
    for (int64_t k = k0; k < k1; ++k) mine += wsum[c0 + k];
    double lo, hi, Q;
    block_scan(mine, sm, &lo, &hi, &Q);
    if (t == 0) Qout[r] = Q;
    if (!(Q > 0.0)) {
        if (t == 0) moves[r].valid = 0;
        return;  // uniform across the block
    }
    const int per_step = rt.kind == 0 ? 1 : 2;  // uniforms per replica and step
    const double uu = u[((int64_t)(*step) * R + r) * per_step];
    double T;
    if (rt.kind == 0) {
        double want = floor(uu * Q);
        want = want < 0.0 ? 0.0 : (want > Q - 1.0 ? Q - 1.0 : want);
        T = want + 1.0;
    } else {
        T = Q * (1.0 - uu);
    }
    // keep T in (0, Q] whatever u holds (also NaN), so exactly one lane owns it
    if (!(T > 0.0)) T = __DBL_DENORM_MIN__;
    if (!(T <= Q)) T = Q;
    if (t == 0) {
        s_chunk = -1;
        s_target = T;
    }
    __syncthreads();
    if (T > lo && T <= hi) {
        double acc = lo;
        int64_t last = -1;
        for (int64_t k = k0; k < k1; ++k) {
            const double w = wsum[c0 + k];
            if (w > 0.0) last = k;
            if (w > 0.0 && T <= acc + w) {
                s_chunk = k;
                s_target = T - acc;
                break;
            }
            acc += w;
        }
        if (s_chunk < 0) {  // rounding: the target lies past the running sum of this lane's chunks
            s_chunk = last;
            s_target = wsum[c0 + last];
        }
    }
    __syncthreads();
    if (s_chunk < 0) {  // not reached for T in (0, Q]; a guard against reading outside the replica
        if (t == 0) moves[r].valid = 0;
        return;
    }
    // within the chunk: kSelLane consecutive slots per lane, added in the same
    // order as in k_b_count
    const int64_t b0 = s_chunk * kSelChunk + (int64_t)t * kSelLane;
    double w[kSelLane], mine2 = 0.0;
    lane_rates(d, rt, b0, w);
#pragma unroll
    for (int k = 0; k < kSelLane; ++k) mine2 += w[k];
    double lo2, hi2, tot2;
    block_scan(mine2, sm, &lo2, &hi2, &tot2);
    const double T2 = s_target < tot2 ? s_target : tot2;  // rounding at the chunk's end
    if (t == 0) s_slot = -1;
    __syncthreads();
    if (T2 > lo2 && T2 <= hi2) {
        double acc = lo2;
        int jl = -1;
#pragma unroll
        for (int k = 0; k < kSelLane; ++k) {
            if (w[k] > 0.0 && jl < 0) {
                if (T2 <= acc + w[k]) jl = k;
            }
            acc += w[k];
        }
        if (jl < 0) {  // rounding: the last slot of this lane with a propensity
#pragma unroll
            for (int k = 0; k < kSelLane; ++k)
                if (w[k] > 0.0) jl = k;
        }
        s_slot = b0 + jl;
    }
    __syncthreads();
    if (t == 0) {
        int64_t slot = s_slot;
        if (slot < 0) {  // rounding: the last slot of the chunk with a propensity
            const int64_t S = d.N * d.K;
            for (int64_t e = s_chunk * kSelChunk + kSelChunk - 1; e >= s_chunk * kSelChunk; --e)
                if (e < S && slot_rate(rt, d.mask[e], rt.kind != 0 ? d.dU[e] : 0.0) > 0.0) {
                    slot = e;
                    break;
                }
        }
        if (slot >= 0)
            prepare_move(d, slot, moves[r]);
        else
            moves[r].valid = 0;  // not reached: the chunk holds a slot with a propensity
    }
}

// U += dU (parts added in order, as the single-context accept does), outputs, next step
__global__ __launch_bounds__(256) void k_b_finish(const MoveDev *__restrict__ moves, int R,
                                                  const double *__restrict__ acc, double *__restrict__ U,
                                                  int32_t *__restrict__ step, int64_t *__restrict__ out_i,
                                                  int64_t *__restrict__ out_site, double *__restrict__ out_dU,
                                                  Rates rt, const double *__restrict__ u,
                                                  const double *__restrict__ Q, double *__restrict__ out_dt)
{
    const int st = *step;
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const MoveDev &m = moves[r];
        // time increment of Alg. 1: -log(xi) / Q with xi = 1 - u in (0, 1]; with no
        // propensity (Q = 0) no event happens: +inf; kind 0 has no rates: NaN
        const int64_t o = (int64_t)st * R + r;
        double dt = __builtin_nan("");
        if (rt.kind != 0) dt = Q[r] > 0.0 ? -log(1.0 - u[2 * o + 1]) / Q[r] : __builtin_inf();
        out_dt[o] = dt;
        double dU = __builtin_nan("");
        int64_t i = -1, site = -1;
        if (m.valid) {
            dU = 0.0;
            for (int k = 0; k < kMoveParts; ++k) dU += acc[(int64_t)r * kMoveParts + k];
            U[r] += dU;
            i = m.i;
            site = m.new_site;
        }
        out_i[o] = i;
        out_site[o] = site;
        out_dU[o] = dU;
    }
    __syncthreads();
    if (threadIdx.x == 0) *step = st + 1;
}

__global__ void k_b_set_step(int32_t *step, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step = v;
}

// zero-charge moves (valid, q = 0) for timing the sweep: they add exact zeros
__global__ void k_b_null_moves(const RepDev *__restrict__ reps, int R, MoveDev *__restrict__ moves)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const double p = 0.3 * reps[r].g.w;
    MoveDev &m = moves[r];
    m.valid = 1;
    m.mv.ox = m.mv.oy = m.mv.oz = m.mv.nx = m.mv.ny = m.mv.nz = p;
    m.mv.q = 0.0;
    m.mv.ogx = m.mv.ogy = m.mv.ogz = m.mv.ngx = m.mv.ngy = m.mv.ngz = 0;
}

}  // namespace

namespace fmmkmc {
// block ranges of one batched phase
struct Phase {
    std::vector<int64_t> base;  // host copy, R + 1
    int64_t *d = nullptr;       // device copy
    int64_t blocks = 0;
};
}  // namespace fmmkmc

struct fmmkmc_batch {
    int R = 0, p = 0, nt = 0, K = 0, device = 0;
    bool mixed = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t aux = nullptr;  // side stream: the F rows run beside the sweep
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<fmmkmc_ctx *> ctx;
    std::vector<int32_t> offsets;
    std::vector<RepDev> host_reps;  // what the device descriptors hold
    std::string err;
    Profiler prof;
    // device state
    RepDev *reps = nullptr;
    MoveDev *moves = nullptr, *null_moves = nullptr;
    double *acc = nullptr, *U = nullptr;
    int32_t *step = nullptr;
    double *wsum = nullptr, *Q = nullptr;  // chunk propensities, total per replica
    std::vector<double *> dU;
    std::vector<uint8_t *> mask;
    Rates rates{0, 1.0, 1.0};
    double *u = nullptr;  // uniforms of the steps: 1 (kind 0) or 2 per replica and step
    int64_t *out_i = nullptr, *out_site = nullptr;
    double *out_dU = nullptr, *out_dt = nullptr;
    int cap_steps = 0;
    // phases
    Phase site, site_lf, site_gen, slot, count, sweep, path, far, cheb_a, cheb_b, coarse;
    Phase coarse_s2;  // every coarse level of the 2x2x2 replicas (per-level mode)
    int slot_tc = 64, sweep_block = 256;
    bool per_level = false;  // replicas keep their local expansions per level (no sweep)
    bool frow = false;       // some replica keeps a per-charge hop table F (periodic, expansion self terms)
    int Lmax = 0;
    int64_t slots_per_step = 0;
    // graph of one step
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int bfail(fmmkmc_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

#define BATCH_GUARD(b, ...)                                                      \
    try {                                                                        \
        __VA_ARGS__                                                              \
    } catch (const HipError &e) {                                                \
        return bfail(b, FMMKMC_EHIP, e.what);                                    \
    } catch (const std::bad_alloc &) {                                           \
        return bfail(b, FMMKMC_ENOMEM, "device or host allocation failed");      \
    }

void set_phase(Phase &ph, const std::vector<int64_t> &blocks_per_rep, hipStream_t s)
{
    const int R = (int)blocks_per_rep.size();
    ph.base.assign(R + 1, 0);
    for (int r = 0; r < R; ++r) ph.base[r + 1] = ph.base[r] + blocks_per_rep[r];
    ph.blocks = ph.base[R];
    dfree(ph.d);
    ph.d = dalloc<int64_t>(R + 1);
    upload(ph.d, ph.base.data(), R + 1, s);
}

void set_sweep_phase(fmmkmc_batch *b)
{
    std::vector<int64_t> nb(b->R);
    for (int r = 0; r < b->R; ++r) nb[r] = (b->ctx[r]->M + b->sweep_block - 1) / b->sweep_block;
    set_phase(b->sweep, nb, b->stream);
}

void set_slot_phase(fmmkmc_batch *b)
{
    std::vector<int64_t> nb(b->R);
    for (int r = 0; r < b->R; ++r) nb[r] = (b->ctx[r]->N + b->slot_tc - 1) / b->slot_tc;
    set_phase(b->slot, nb, b->stream);
}

// the phases of one step, in order
void record_step(fmmkmc_batch *b)
{
    const hipStream_t s = b->stream;
    const int R = b->R;
    if (b->per_level) {
        launch_b_coarse(b->prof, s, b->reps, R, b->coarse.d, b->coarse.blocks, b->p);
        if (b->coarse_s2.blocks)
            launch_b_coarse_s2(b->prof, s, b->reps, R, b->coarse_s2.d, b->coarse_s2.blocks, b->p);
    }
    launch_b_site(b->prof, s, b->reps, R, b->site.d, b->site.blocks, b->site_lf.d, b->site_lf.blocks, b->site_gen.d,
                  b->site_gen.blocks, b->p, b->mixed);
    launch_b_slot(b->prof, s, b->reps, R, b->slot.d, b->slot.blocks, b->slot_tc);
    launch_prof(b->prof, s, "b_count", k_b_count, dim3((unsigned)b->count.blocks), dim3(256), 0, b->reps, R,
                b->count.d, b->rates, b->wsum);
    launch_prof(b->prof, s, "b_select", k_b_select, dim3((unsigned)R), dim3(256), 0, b->reps, R, b->count.d,
                b->wsum, b->rates, b->u, b->step, b->moves, b->Q);
    // the part of the move's dU that reads the fine-level expansions, before the sweep
    launch_b_move_dU(b->prof, s, b->reps, R, b->moves, b->acc, b->nt, 0, 1, b->per_level ? b->Lmax - 1 : 1);
    // beside the sweep, on the side stream: the rest of the move's dU (cell
    // lists and far-field tables, before the bookkeeping and the far-field
    // update change them), the F rows (they depend only on the moves), the
    // multipole paths, the bookkeeping and the far field; none of it touches
    // the fine-level expansions or what the sweep reads
    HIPCHK(hipEventRecord(b->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(b->aux, b->ev_fork, 0));
    launch_b_move_dU(b->prof, b->aux, b->reps, R, b->moves, b->acc, b->nt, 1, kMoveParts - 1, 1);
    if (b->frow) launch_b_frow(b->prof, b->aux, b->reps, R, b->moves, b->nt, b->K);  // no-ops without an F table
    launch_b_path(b->prof, b->aux, b->reps, R, b->path.d, b->path.blocks, b->moves);
    launch_b_book(b->prof, b->aux, b->reps, R, b->moves);
    launch_b_far(b->prof, b->aux, b->reps, R, b->far.d, b->far.blocks, b->cheb_a.d, b->cheb_a.blocks, b->cheb_b.d,
                 b->cheb_b.blocks, b->moves);
    HIPCHK(hipEventRecord(b->ev_join, b->aux));
    if (b->per_level)
        launch_b_levels(b->prof, s, b->reps, R, b->p, b->moves, b->Lmax, 2);
    else
        launch_b_sweep(b->prof, s, b->reps, R, b->sweep.d, b->sweep.blocks, b->p, b->moves, b->sweep_block);
    HIPCHK(hipStreamWaitEvent(s, b->ev_join, 0));
    launch_prof(b->prof, s, "b_finish", k_b_finish, dim3(1), dim3(256), 0, (const MoveDev *)b->moves, R,
                (const double *)b->acc, b->U, b->step, b->out_i, b->out_site, b->out_dU, b->rates,
                (const double *)b->u, (const double *)b->Q, b->out_dt);
}

void drop_graph(fmmkmc_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void capture(fmmkmc_batch *b)
{
    drop_graph(b);
    const bool was = b->prof.on;
    b->prof.on = false;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
        record_step(b);
    } catch (...) {
        (void)hipStreamEndCapture(b->stream, &g);  // leave the stream usable
        if (g) (void)hipGraphDestroy(g);
        b->prof.on = was;
        throw;
    }
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->prof.on = was;
    HIPCHK(e);
    b->graph = g;
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
}

void ensure_steps(fmmkmc_batch *b, int n_steps)
{
    if (n_steps <= b->cap_steps) return;
    HIPCHK(hipStreamSynchronize(b->stream));
    const int cap = std::max(n_steps, 2 * b->cap_steps);
    const size_t m = (size_t)cap * b->R;
    dfree(b->u);
    dfree(b->out_i);
    dfree(b->out_site);
    dfree(b->out_dU);
    dfree(b->out_dt);
    b->u = dalloc<double>(2 * m);
    b->out_i = dalloc<int64_t>(m);
    b->out_site = dalloc<int64_t>(m);
    b->out_dU = dalloc<double>(m);
    b->out_dt = dalloc<double>(m);
    b->cap_steps = cap;
    drop_graph(b);  // the captured launches hold the old pointers
}

void release_batch(fmmkmc_batch *b)
{
    drop_graph(b);
    dfree(b->reps);
    dfree(b->moves);
    dfree(b->null_moves);
    dfree(b->acc);
    dfree(b->U);
    dfree(b->step);
    dfree(b->wsum);
    dfree(b->Q);
    for (auto &p : b->dU) dfree(p);
    for (auto &p : b->mask) dfree(p);
    dfree(b->u);
    dfree(b->out_i);
    dfree(b->out_site);
    dfree(b->out_dU);
    dfree(b->out_dt);
    for (Phase *ph : {&b->site, &b->site_lf, &b->site_gen, &b->slot, &b->count, &b->sweep, &b->path, &b->far,
                      &b->cheb_a, &b->cheb_b, &b->coarse, &b->coarse_s2})
        dfree(ph->d);
    for (auto &pd : b->prof.pending) {
        (void)hipEventDestroy(pd.a);
        (void)hipEventDestroy(pd.b);
    }
    b->prof.pending.clear();
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->aux) (void)hipStreamDestroy(b->aux);
    b->ev_fork = b->ev_join = nullptr;
    b->aux = nullptr;
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    b->stream = nullptr;
    b->own_stream = false;
}

RepDev make_rep(const fmmkmc_ctx *c, int K, double *dU, uint8_t *mask)
{
    RepDev d{};
    d.g = make_geo(c);
    d.M = c->M;
    d.N = c->N;
    d.L = c->L;
    d.p = c->p;
    d.nt = c->nt;
    d.K = K;
    d.s2 = c->s2 ? 1 : 0;
    d.cap = c->cap;
    d.kmul = (uint32_t)(((uint64_t)1 << 32) / (uint64_t)K);
    d.psi = c->psi_lv[c->L];
    d.psi32 = c->prec == FMMKMC_MIXED ? c->psi32 : nullptr;
    d.phi_lv = c->d_phi_ptrs;
    d.psi_lv = c->d_psi_ptrs;
    d.phicoarse = c->phicoarse;
    d.x = c->x;
    d.y = c->y;
    d.z = c->z;
    d.q = c->q;
    d.cell = c->cell;
    d.slot = c->slot;
    d.site = c->site;
    d.cnt = c->cell_cnt;
    d.slots = c->cell_slots;
    d.rank_of = c->rank_of;
    d.site_charge = c->site_charge;
    d.site_rank = c->site_rank;
    d.qsite = c->qsite;
    d.qsite32 = c->qsite32;
    d.cell_rng = c->cell_rng;
    d.phisite = c->phisite;
    d.order = c->order;
    d.ijk_r = c->ijk_r;
    d.q_r = c->q_r;
    d.phi_r = c->phi_r;
    d.F = (c->bc == FMMKMC_PERIODIC && !c->self_exact) ? c->F : nullptr;
    d.Fhop = (c->bc == FMMKMC_PERIODIC && c->self_exact) ? c->Fhop : nullptr;
    d.frow_w = c->frow_w;
    d.offsets = c->d_offsets;
    d.dU = dU;
    d.mask = mask;
    d.R = c->far.R;
    d.GR = c->far.GR;
    d.Kf = c->far.K;
    d.H = c->far.H;
    d.C = c->far.C;
    d.A = c->far.A;
    d.Bz = c->far.Bz;
    d.Tax = c->far.Tax;
    d.sigma = c->far.sigma;
    d.cz = c->far.cz;
    d.ncz = c->far.ncz;
    return d;
}

// A context proposed with other hop offsets since the batch was built has a new
// hop table: rebuild it for the batch's offsets and refresh the descriptors
// (the step graph holds only the descriptor array, whose address is fixed).
void sync_descriptors(fmmkmc_batch *b)
{
    bool changed = false;
    for (int r = 0; r < b->R; ++r) {
        fmmkmc_ctx *c = b->ctx[r];
        if (c->F_offsets != b->offsets) {
            const int rc = fmmkmc_propose_lattice(c, b->K, b->offsets.data(), b->dU[r], b->mask[r]);
            if (rc != FMMKMC_OK) throw HipError{"proposal pass of replica " + std::to_string(r) + ": " + c->err};
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        const RepDev d = make_rep(c, b->K, b->dU[r], b->mask[r]);
        if (std::memcmp(&d, &b->host_reps[r], sizeof(RepDev)) != 0) {
            b->host_reps[r] = d;
            changed = true;
        }
    }
    if (changed) {
        upload(b->reps, b->host_reps.data(), b->R, b->stream);
        HIPCHK(hipStreamSynchronize(b->stream));
    }
}

// median of the timed launches of fn (events on the batch stream)
template <typename Fn>
float time_launches(fmmkmc_batch *b, int rounds, Fn fn)
{
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    fn();  // warm-up
    std::vector<float> t;
    for (int k = 0; k < rounds; ++k) {
        HIPCHK(hipEventRecord(e0, b->stream));
        fn();
        HIPCHK(hipEventRecord(e1, b->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        t.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

extern "C" {

int fmmkmc_batch_create(int n, fmmkmc_ctx *const *ctx, int K, const int32_t *offsets, void *stream,
                        fmmkmc_batch **out)
{
    if (!out) return FMMKMC_EINVAL;
    *out = nullptr;
    if (n < 1 || !ctx || !offsets || K < 1 || K > kMaxHops) return FMMKMC_EINVAL;
    for (int k = 0; k < 3 * K; ++k)
        if (offsets[k] < -1 || offsets[k] > 1) return FMMKMC_EINVAL;
    for (int r = 0; r < n; ++r) {
        const fmmkmc_ctx *c = ctx[r];
        if (!c || c->lat_n <= 0) return FMMKMC_EINVAL;
        if (!c->initialised) return FMMKMC_ESTATE;
        if (c->p != ctx[0]->p || c->prec != ctx[0]->prec || c->device != ctx[0]->device) return FMMKMC_EINVAL;
        if (c->N * (int64_t)K >= ((int64_t)1 << 32)) return FMMKMC_EINVAL;
        if (c->per_level != ctx[0]->per_level) return FMMKMC_EINVAL;
    }
    fmmkmc_batch *b = new (std::nothrow) fmmkmc_batch();
    if (!b) return FMMKMC_ENOMEM;
    b->R = n;
    b->p = ctx[0]->p;
    b->nt = ctx[0]->nt;
    b->K = K;
    b->device = ctx[0]->device;
    b->mixed = ctx[0]->prec == FMMKMC_MIXED;
    b->per_level = ctx[0]->per_level != 0;
    for (int r = 0; r < n; ++r) {
        b->Lmax = std::max(b->Lmax, ctx[r]->L);
        if (ctx[r]->bc == FMMKMC_PERIODIC && !ctx[r]->self_exact) b->frow = true;
    }
    b->stream = (hipStream_t)stream;
    b->ctx.assign(ctx, ctx + n);
    b->offsets.assign(offsets, offsets + 3 * K);
    try {
        HIPCHK(hipSetDevice(b->device));
        if (!b->stream) {
            // graphs cannot be captured on the legacy null stream: use a stream of our own
            HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            b->own_stream = true;
        }
        const hipStream_t s = b->stream;
        HIPCHK(hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
        std::vector<RepDev> reps(n);
        std::vector<double> U(n);
        b->dU.assign(n, nullptr);
        b->mask.assign(n, nullptr);
        for (int r = 0; r < n; ++r) {
            fmmkmc_ctx *c = ctx[r];
            b->dU[r] = dalloc<double>((size_t)c->N * K);
            b->mask[r] = dalloc<uint8_t>((size_t)c->N * K);
            // one ordinary proposal pass builds the context's hop table for these offsets
            const int rc = fmmkmc_propose_lattice(c, K, offsets, b->dU[r], b->mask[r]);
            if (rc != FMMKMC_OK) throw HipError{"proposal pass of replica " + std::to_string(r) + ": " + c->err};
            HIPCHK(hipStreamSynchronize(c->stream));
            reps[r] = make_rep(c, K, b->dU[r], b->mask[r]);
            U[r] = c->U;
            b->slots_per_step += c->N * K;
        }
        b->reps = dalloc<RepDev>(n);
        upload(b->reps, reps.data(), n, s);
        b->host_reps = reps;
        b->moves = dalloc<MoveDev>(n);
        b->null_moves = dalloc<MoveDev>(n);
        b->acc = dalloc<double>((size_t)n * kMoveParts);
        b->U = dalloc<double>(n);
        upload(b->U, U.data(), n, s);
        b->step = dalloc<int32_t>(1);
        // phase block tables
        std::vector<int64_t> nsite(n), nsite_lf(n), nsite_gen(n), ncount(n), npath(n), nfar(n), na(n), nb(n),
            ncoarse(n);
        for (int r = 0; r < n; ++r) {
            const fmmkmc_ctx *c = ctx[r];
            const int64_t ns = (int64_t)c->lat_n * c->lat_n * c->lat_n;
            const int q = c->p + 1;
            nsite[r] = c->s2 ? (c->M + 255) / 256 : 0;
            nsite_lf[r] = c->s2 ? 0 : general_site_blocks(c->lat_n, c->nc);
            nsite_gen[r] = c->s2 ? 0 : general_site_blocks(c->lat_n, c->nc);
            ncount[r] = (c->N * K + kSelChunk - 1) / kSelChunk;
            npath[r] = ((int64_t)c->L * (q * (q + 1) / 2) + 255) / 256;
            const bool per = c->bc == FMMKMC_PERIODIC;
            nfar[r] = per ? (c->nt + c->far.ncz + 15) / 16 : 0;
            na[r] = per ? ((int64_t)c->lat_n * q * q + 255) / 256 : 0;
            nb[r] = per ? ((int64_t)c->lat_n * c->lat_n * q + 255) / 256 : 0;
            ncoarse[r] = (c->phicoarse && !c->s2) ? (ns + 255) / 256 : 0;
        }
        set_phase(b->coarse, ncoarse, s);
        {
            // 2x2x2 replicas: every coarse level in one launch
            std::vector<int64_t> nc2(n, 0);
            for (int r = 0; r < n; ++r) {
                const fmmkmc_ctx *c = ctx[r];
                const int lstart = c->bc == FMMKMC_PERIODIC ? 2 : 3;
                if (c->phicoarse && c->s2) nc2[r] = coarse_s2_replica_blocks(c->L, lstart);
            }
            set_phase(b->coarse_s2, nc2, s);
        }
        set_phase(b->site, nsite, s);
        set_phase(b->site_lf, nsite_lf, s);
        set_phase(b->site_gen, nsite_gen, s);
        set_phase(b->count, ncount, s);
        set_phase(b->path, npath, s);
        set_phase(b->far, nfar, s);
        set_phase(b->cheb_a, na, s);
        set_phase(b->cheb_b, nb, s);
        set_slot_phase(b);
        set_sweep_phase(b);
        b->wsum = dalloc<double>(b->count.blocks);
        b->Q = dalloc<double>(n);
        hipLaunchKernelGGL(k_b_null_moves, dim3((n + 63) / 64), dim3(64), 0, s, (const RepDev *)b->reps, n,
                           b->null_moves);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
    } catch (const HipError &e) {
        create_error() = e.what;
        release_batch(b);
        delete b;
        return FMMKMC_EHIP;
    } catch (const std::bad_alloc &) {
        create_error() = "device or host allocation failed";
        release_batch(b);
        delete b;
        return FMMKMC_ENOMEM;
    }
    *out = b;
    return FMMKMC_OK;
}

int fmmkmc_batch_set_rates(fmmkmc_batch *b, int kind, double nu, double beta)
{
    if (!b) return FMMKMC_EINVAL;
    if (kind < 0 || kind > 2) return bfail(b, FMMKMC_EINVAL, "rate kind must be 0, 1 or 2");
    if (kind != 0 && !(nu > 0.0 && std::isfinite(nu) && beta >= 0.0 && std::isfinite(beta)))
        return bfail(b, FMMKMC_EINVAL, "need nu > 0 and beta >= 0, both finite");
    BATCH_GUARD(b, {
        HIPCHK(hipSetDevice(b->device));
        HIPCHK(hipStreamSynchronize(b->stream));
        b->rates = Rates{kind, nu, beta};
        drop_graph(b);  // the captured launches hold the old rate arguments
        return FMMKMC_OK;
    })
}

int fmmkmc_batch_step(fmmkmc_batch *b, int n_steps, const double *u, int64_t *moved, int64_t *site, double *dU,
                      double *dt)
{
    if (!b) return FMMKMC_EINVAL;
    if (n_steps < 0 || (n_steps > 0 && !u)) return bfail(b, FMMKMC_EINVAL, "need n_steps >= 0 and u");
    if (n_steps == 0) return FMMKMC_OK;
    BATCH_GUARD(b, {
        HIPCHK(hipSetDevice(b->device));
        for (fmmkmc_ctx *c : b->ctx) HIPCHK(hipStreamSynchronize(c->stream));
        sync_descriptors(b);
        ensure_steps(b, n_steps);
        const hipStream_t s = b->stream;
        const size_t m = (size_t)n_steps * b->R;
        const size_t nu = b->rates.kind == 0 ? 1 : 2;
        HIPCHK(hipMemcpyAsync(b->u, u, sizeof(double) * m * nu, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_b_set_step, dim3(1), dim3(64), 0, s, b->step, 0);
        HIPCHK(hipGetLastError());
        if (b->prof.on) {
            for (int k = 0; k < n_steps; ++k) record_step(b);
        } else {
            if (!b->exec) capture(b);
            for (int k = 0; k < n_steps; ++k) HIPCHK(hipGraphLaunch(b->exec, s));
        }
        HIPCHK(hipGetLastError());
        if (moved) HIPCHK(hipMemcpyAsync(moved, b->out_i, sizeof(int64_t) * m, hipMemcpyDeviceToDevice, s));
        if (site) HIPCHK(hipMemcpyAsync(site, b->out_site, sizeof(int64_t) * m, hipMemcpyDeviceToDevice, s));
        if (dU) HIPCHK(hipMemcpyAsync(dU, b->out_dU, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
        if (dt) HIPCHK(hipMemcpyAsync(dt, b->out_dt, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
        std::vector<double> U(b->R);
        HIPCHK(hipMemcpyAsync(U.data(), b->U, sizeof(double) * b->R, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int r = 0; r < b->R; ++r) {
            b->ctx[r]->U = U[r];
            b->ctx[r]->dev_ahead = true;
        }
        return FMMKMC_OK;
    })
}

int fmmkmc_batch_proposals(fmmkmc_batch *b, int r, double *dU, uint8_t *mask)
{
    if (!b) return FMMKMC_EINVAL;
    if (r < 0 || r >= b->R || !dU) return bfail(b, FMMKMC_EINVAL, "bad replica or dU");
    BATCH_GUARD(b, {
        HIPCHK(hipSetDevice(b->device));
        const size_t m = (size_t)b->ctx[r]->N * b->K;
        HIPCHK(hipMemcpyAsync(dU, b->dU[r], sizeof(double) * m, hipMemcpyDeviceToDevice, b->stream));
        if (mask) HIPCHK(hipMemcpyAsync(mask, b->mask[r], m, hipMemcpyDeviceToDevice, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        return FMMKMC_OK;
    })
}

int fmmkmc_batch_tune(fmmkmc_batch *b, int rounds)
{
    if (!b) return FMMKMC_EINVAL;
    if (rounds < 1) return bfail(b, FMMKMC_EINVAL, "rounds must be >= 1");
    BATCH_GUARD(b, {
        HIPCHK(hipSetDevice(b->device));
        for (fmmkmc_ctx *c : b->ctx) HIPCHK(hipStreamSynchronize(c->stream));
        const hipStream_t s = b->stream;
        const bool was = b->prof.on;
        b->prof.on = false;
        // slot gather: charges per block (reads the site potentials of the current configuration)
        launch_b_site(b->prof, s, b->reps, b->R, b->site.d, b->site.blocks, b->site_lf.d, b->site_lf.blocks,
                      b->site_gen.d, b->site_gen.blocks, b->p, b->mixed);
        float best = 0;
        int best_tc = b->slot_tc;
        for (int tc : {32, 64, 128}) {
            b->slot_tc = tc;
            set_slot_phase(b);
            const float t = time_launches(b, rounds, [&] {
                launch_b_slot(b->prof, s, b->reps, b->R, b->slot.d, b->slot.blocks, b->slot_tc);
            });
            if (tc == 32 || t < best) {
                best = t;
                best_tc = tc;
            }
        }
        b->slot_tc = best_tc;
        set_slot_phase(b);
        // sweep: threads per block, timed with zero-charge moves (they leave every expansion unchanged)
        int best_blk = b->sweep_block;
        for (int blk : {128, 256}) {
            if (b->per_level) break;  // no sweep
            b->sweep_block = blk;
            set_sweep_phase(b);
            const float t = time_launches(b, rounds, [&] {
                launch_b_sweep(b->prof, s, b->reps, b->R, b->sweep.d, b->sweep.blocks, b->p, b->null_moves,
                               b->sweep_block);
            });
            if (blk == 128 || t < best) {
                best = t;
                best_blk = blk;
            }
        }
        b->sweep_block = best_blk;
        set_sweep_phase(b);
        HIPCHK(hipStreamSynchronize(s));
        b->prof.on = was;
        drop_graph(b);
        return FMMKMC_OK;
    })
}

int fmmkmc_batch_info(fmmkmc_batch *b, int64_t *slots_per_step, int *slot_tile, int *sweep_block)
{
    if (!b) return FMMKMC_EINVAL;
    if (slots_per_step) *slots_per_step = b->slots_per_step;
    if (slot_tile) *slot_tile = b->slot_tc;
    if (sweep_block) *sweep_block = b->sweep_block;
    return FMMKMC_OK;
}

int fmmkmc_batch_set_profiling(fmmkmc_batch *b, int on)
{
    if (!b) return FMMKMC_EINVAL;
    BATCH_GUARD(b, {
        HIPCHK(hipStreamSynchronize(b->stream));
        b->prof.resolve();
        b->prof.total.clear();
        b->prof.on = on != 0;
        return FMMKMC_OK;
    })
}

int fmmkmc_batch_kernel_time(fmmkmc_batch *b, const char *name, double *ms, int64_t *launches)
{
    if (!b || !name) return FMMKMC_EINVAL;
    b->prof.resolve();
    auto it = b->prof.total.find(name);
    if (ms) *ms = it == b->prof.total.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == b->prof.total.end() ? 0 : it->second.second;
    return FMMKMC_OK;
}

const char *fmmkmc_batch_last_error(fmmkmc_batch *b)
{
    if (!b) return create_error().c_str();
    return b->err.c_str();
}

int fmmkmc_batch_destroy(fmmkmc_batch *b)
{
    if (!b) return FMMKMC_OK;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    release_batch(b);
    delete b;
    return FMMKMC_OK;
}

}  // extern "C"
