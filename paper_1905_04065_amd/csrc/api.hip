// C-ABI of the fmmkmc library (declared in include/fmmkmc.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hostutil.hpp"
#include "kernels.hpp"
#include "tables.hpp"

using namespace fmmkmc;

// ---- work memory of the allocation-free generic proposal call ---------------
// fmmkmc_propose_noalloc() keeps its per-slot work (wrapped target, potentials at
// the target and at the charge, far-field change, status word, charge index:
// 72 bytes per slot) in this file-scope device array instead of memory allocated
// per call.  Every GPU the library runs on holds one copy until the process
// ends; all calls on that GPU share it, so such calls must not overlap on one
// GPU.  Host code never uses the array's name as an address: each device's copy
// is looked up once (hipGetSymbolAddress, at the first context created on that
// device) and the kernels get that address.
constexpr int64_t kNoAllocSlots = (int64_t)1 << 18;
constexpr int64_t kNoAllocBytes = 72 * kNoAllocSlots;  // 18 MiB
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// this device's copy of `scratch` (the device must be current); nullptr if the
// device ordinal is beyond the table
void *device_scratch(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

// context-owned work buffer of at least `bytes` (grown on demand)
void *work_buffer(fmmkmc_ctx *c, size_t bytes)
{
    if (c->scr_bytes < bytes) {
        HIPCHK(hipStreamSynchronize(c->stream));
        dfree(c->scr);
        c->scr = dalloc<double>((bytes + 7) / 8);
        c->scr_bytes = ((bytes + 7) / 8) * 8;
    }
    return c->scr;
}

double lattice_h(const fmmkmc_ctx *c) { return c->a / c->lat_n; }

// lattice index of a position, -1 if it is not a site
int64_t site_of(const fmmkmc_ctx *c, const double *p)
{
    const int n = c->lat_n;
    const double h = lattice_h(c);
    int idx[3];
    for (int d = 0; d < 3; ++d) {
        const double u = p[d] / h - 0.5;
        const double r = std::nearbyint(u);
        if (r < 0 || r >= n) return -1;
        if ((r + 0.5) * h != p[d]) return -1;
        idx[d] = (int)r;
    }
    return ((int64_t)idx[0] * n + idx[1]) * n + idx[2];
}

void fine_of(const fmmkmc_ctx *c, const double *p, int g[3])
{
    const double w = c->a / c->nc;
    for (int d = 0; d < 3; ++d) g[d] = fine_coord(p[d], w, c->nc);
}

// index of a lattice site (lattice order) in the device's site order
int64_t site_order(const fmmkmc_ctx *c, int64_t lat)
{
    if (!c->s2) return lat;
    const int n = c->lat_n;
    return s2_site(c->nc, (int)(lat / ((int64_t)n * n)), (int)((lat / n) % n), (int)(lat % n));
}

int32_t pack_ijk(const fmmkmc_ctx *c, int64_t lat)
{
    const int n = c->lat_n;
    const int i = (int)(lat / ((int64_t)n * n)), j = (int)((lat / n) % n), k = (int)(lat % n);
    return (int32_t)((i << 20) | (j << 10) | k);
}

}  // namespace

// Host mirrors of a context whose device state was advanced by batched steps
// (the batch moves charges on the device only): download what the
// single-context accept validates against.
void refresh_mirrors(fmmkmc_ctx *c)
{
    if (!c->dev_ahead) return;
    const int64_t n = c->N;
    const hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(c->hx.data(), c->x, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->hy.data(), c->y, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->hz.data(), c->z, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->hcell.data(), c->cell, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->hslot.data(), c->slot, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->hcnt.data(), c->cell_cnt, sizeof(int32_t) * c->M, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->hslots.data(), c->cell_slots, sizeof(int32_t) * c->M * c->cap, hipMemcpyDeviceToHost,
                          s));
    if (c->lat_n > 0) {
        HIPCHK(hipMemcpyAsync(c->hsite.data(), c->site, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::fill(c->hsite_charge.begin(), c->hsite_charge.end(), -1);
        for (int64_t i = 0; i < n; ++i) c->hsite_charge[c->hsite[i]] = (int32_t)i;
    }
    HIPCHK(hipStreamSynchronize(s));
    c->dev_ahead = false;
}

namespace {

void release(fmmkmc_ctx *c)
{
    dfree(c->x);
    dfree(c->y);
    dfree(c->z);
    dfree(c->q);
    dfree(c->cell);
    dfree(c->slot);
    dfree(c->site);
    dfree(c->cell_cnt);
    dfree(c->cell_slots);
    dfree(c->site_charge);
    dfree(c->order);
    dfree(c->q_r);
    dfree(c->ijk_r);
    dfree(c->qsite);
    dfree(c->qsite32);
    dfree(c->cell_rng);
    for (auto &p : c->phi_lv) dfree(p);
    for (auto &p : c->psi_lv) dfree(p);
    dfree(c->d_phi_ptrs);
    dfree(c->d_psi_ptrs);
    dfree(c->phicoarse);
    dfree(c->psi32);
    dfree(c->phisite);
    for (auto &p : c->m2m) dfree(p);
    for (auto &p : c->l2l) dfree(p);
    dfree(c->m2l);
    dfree(c->m2l_index);
    dfree(c->scale);
    dfree(c->site_rank);
    dfree(c->phi_r);
    dfree(c->far.H);
    dfree(c->far.R);
    dfree(c->far.GR);
    dfree(c->far.cz);
    dfree(c->far.A);
    dfree(c->far.C);
    dfree(c->far.Bz);
    dfree(c->far.Tax);
    dfree(c->far.sigma);
    c->far.K = nullptr;  // alias of phi_lv[1]
    dfree(c->F);
    dfree(c->Fhop);
    dfree(c->frow_w);
    dfree(c->d_offsets);
    dfree(c->scr);
    dfree(c->flags);
    dfree(c->red);
    dfree(c->iota);
    dfree(c->acc_buf);
    dfree(c->rank_of);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    c->ev_fork = c->ev_join = nullptr;
    c->aux = nullptr;
    for (auto &pd : c->prof.pending) {
        (void)hipEventDestroy(pd.a);
        (void)hipEventDestroy(pd.b);
    }
    c->prof.pending.clear();
}

void build_operators(fmmkmc_ctx *c)
{
    const int p = c->p, nt = c->nt, L = c->L;
    std::vector<double> mat((size_t)nt * nt), tr((size_t)nt * nt);
    auto transpose = [&](const double *src, double *dst) {
        for (int k = 0; k < nt; ++k)
            for (int n = 0; n < nt; ++n) dst[(size_t)n * nt + k] = src[(size_t)k * nt + n];
    };
    c->m2m.assign(L + 1, nullptr);
    c->l2l.assign(L + 1, nullptr);
    std::vector<double> all((size_t)8 * nt * nt);
    for (int l = 1; l <= L; ++l) {
        const double wc = c->a / (1 << l);  // child width (level l + 1)
        if (l <= L - 1) {
            for (int ch = 0; ch < 8; ++ch) {
                const int ox = ch >> 2, oy = (ch >> 1) & 1, oz = ch & 1;
                build_m2m(p, (ox - 0.5) * wc, (oy - 0.5) * wc, (oz - 0.5) * wc, mat.data());
                transpose(mat.data(), all.data() + (size_t)ch * nt * nt);
            }
            c->m2m[l] = dalloc<double>(all.size());
            upload(c->m2m[l], all.data(), all.size(), c->stream);
            HIPCHK(hipStreamSynchronize(c->stream));
        }
        if (l >= 2) {
            const double w = c->a / (1 << (l - 1));  // width at level l
            for (int ch = 0; ch < 8; ++ch) {
                const int ox = ch >> 2, oy = (ch >> 1) & 1, oz = ch & 1;
                build_l2l(p, (ox - 0.5) * w, (oy - 0.5) * w, (oz - 0.5) * w, mat.data());
                transpose(mat.data(), all.data() + (size_t)ch * nt * nt);
            }
            c->l2l[l] = dalloc<double>(all.size());
            upload(c->l2l[l], all.data(), all.size(), c->stream);
            HIPCHK(hipStreamSynchronize(c->stream));
        }
    }
    // M2L for unit width, keyed by d = target - source in {-3..3}^3 \ {-1..1}^3
    std::vector<int32_t> index(343, -1);
    std::vector<double> m2l;
    int o = 0;
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz) {
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1) continue;
                index[(dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)] = o++;
            }
    m2l.resize((size_t)o * nt * nt);
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz) {
                const int id = index[(dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)];
                if (id < 0) continue;
                build_m2l(p, dx, dy, dz, mat.data());
                transpose(mat.data(), m2l.data() + (size_t)id * nt * nt);
            }
    c->m2l = dalloc<double>(m2l.size());
    upload(c->m2l, m2l.data(), m2l.size(), c->stream);
    c->m2l_index = dalloc<int32_t>(343);
    upload(c->m2l_index, index.data(), 343, c->stream);
    // per-level scales of the unit-width M2L: input w^-deg(n), output w^-(deg(k)+1)
    std::vector<double> sc((size_t)2 * (L + 1) * nt, 0.0);
    for (int l = 1; l <= L; ++l) {
        const double w = c->a / (1 << (l - 1));
        for (int n = 0; n <= p; ++n)
            for (int k = n * n; k < (n + 1) * (n + 1); ++k) {
                sc[(size_t)(2 * l) * nt + k] = std::pow(w, -n);
                sc[(size_t)(2 * l + 1) * nt + k] = std::pow(w, -(n + 1.0));
            }
    }
    c->scale = dalloc<double>(sc.size());
    upload(c->scale, sc.data(), sc.size(), c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
}

void build_far(fmmkmc_ctx *c)
{
    const int p = c->p, nt = c->nt, q = p + 1, ncheb = q * q * q;
    std::vector<double> R((size_t)nt * nt), RT((size_t)nt * nt);
    build_far_operator(p, c->a, R.data());
    for (int k = 0; k < nt; ++k)
        for (int n = 0; n < nt; ++n) RT[(size_t)n * nt + k] = R[(size_t)k * nt + n];
    c->far.R = dalloc<double>(RT.size());
    upload(c->far.R, RT.data(), RT.size(), c->stream);
    // C = G H = (G R) K: fold R into the Chebyshev map once; only the rows of
    // total degree a + b + c <= p are nonzero; stored [n][row]
    std::vector<double> G((size_t)ncheb * nt);
    build_cheb_map(p, c->a, G.data());
    std::vector<int32_t> cz;
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
            for (int cc = 0; cc < q; ++cc)
                if (a + b + cc <= p) cz.push_back((a * q + b) * q + cc);
    const int ncz = (int)cz.size();
    std::vector<double> GRT((size_t)nt * ncz, 0.0);
    for (int r = 0; r < ncz; ++r) {
        const double *g = &G[(size_t)cz[r] * nt];
        for (int n = 0; n < nt; ++n) {
            double s = 0.0;
            for (int k = 0; k < nt; ++k) s += g[k] * R[(size_t)k * nt + n];
            GRT[(size_t)n * ncz + r] = s;
        }
    }
    c->far.ncz = ncz;
    c->far.GR = dalloc<double>(GRT.size());
    upload(c->far.GR, GRT.data(), GRT.size(), c->stream);
    c->far.cz = dalloc<int32_t>(ncz);
    upload(c->far.cz, cz.data(), ncz, c->stream);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->far.C = dalloc<double>((size_t)q * q * q);
    HIPCHK(hipMemsetAsync(c->far.C, 0, sizeof(double) * q * q * q, c->stream));
    c->far.H = dalloc<double>(nt);
    c->far.K = c->phi_lv[1];
    if (c->lat_n > 0) {
        const int n = c->lat_n;
        std::vector<double> Tax((size_t)n * q);
        const double h = lattice_h(c);
        for (int i = 0; i < n; ++i) {
            const double xi = ((i + 0.5) * h - 0.5 * c->a) / (0.5 * c->a);
            double t0 = 1.0, t1 = xi;
            for (int aa = 0; aa < q; ++aa) {
                double v = aa == 0 ? 1.0 : (aa == 1 ? xi : 2.0 * xi * t1 - t0);
                if (aa >= 2) {
                    t0 = t1;
                    t1 = v;
                }
                Tax[(size_t)i * q + aa] = v;
            }
        }
        c->far.Tax = dalloc<double>(Tax.size());
        upload(c->far.Tax, Tax.data(), Tax.size(), c->stream);
        c->far.Bz = dalloc<double>((size_t)n * n * q);
        c->far.A = dalloc<double>((size_t)n * q * q);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
}

int create_impl(const fmmkmc_params *prm, int64_t n, const double *xyz, const double *qv, fmmkmc_ctx *c)
{
    if (!prm || !xyz || !qv) return fail(c, FMMKMC_EINVAL, "null argument");
    if (!(prm->a > 0)) return fail(c, FMMKMC_EINVAL, "box side a must be > 0");
    if (prm->bc != FMMKMC_FREE && prm->bc != FMMKMC_PERIODIC) return fail(c, FMMKMC_EINVAL, "bc must be 0 or 1");
    const int minL = prm->bc == FMMKMC_PERIODIC ? 3 : 2;
    if (prm->levels < minL || prm->levels > kMaxLevels)
        return fail(c, FMMKMC_EINVAL, "levels out of range (free >= 2, periodic >= 3, <= 10)");
    if (prm->order < 1 || prm->order > kMaxOrder) return fail(c, FMMKMC_EINVAL, "order must be in 1..16");
    if (prm->precision != FMMKMC_FP64 && prm->precision != FMMKMC_MIXED)
        return fail(c, FMMKMC_EINVAL, "precision must be 0 or 1");
    if (prm->lattice_n < 0 || prm->cell_capacity < 0) return fail(c, FMMKMC_EINVAL, "negative lattice_n/capacity");
    if (n < 1 || n > (int64_t)1 << 30) return fail(c, FMMKMC_EINVAL, "charge count out of range");
    c->a = prm->a;
    c->bc = prm->bc;
    c->L = prm->levels;
    c->p = prm->order;
    c->nt = nterms(c->p);
    c->prec = prm->precision;
    if (prm->self_image != 0 && prm->self_image != 1) return fail(c, FMMKMC_EINVAL, "self_image must be 0 or 1");
    c->self_exact = (prm->bc == FMMKMC_PERIODIC && prm->self_image == 1) ? 1 : 0;
    if (prm->per_level != 0 && prm->per_level != 1) return fail(c, FMMKMC_EINVAL, "per_level must be 0 or 1");
    c->per_level = prm->per_level;
    c->lat_n = prm->lattice_n;
    c->device = prm->device;
    c->stream = (hipStream_t)prm->stream;
    c->N = n;
    c->nc = 1 << (c->L - 1);
    c->M = (int64_t)c->nc * c->nc * c->nc;
    if (c->lat_n > 0) {
        c->h = lattice_h(c);
        if (c->lat_n > kMaxLattice) return fail(c, FMMKMC_EINVAL, "lattice_n must be <= 1024");
    }
    HIPCHK(hipSetDevice(c->device));
    (void)device_scratch(c->device);  // resolve this device's work array once, at set-up
    HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    // host copies; periodic positions wrapped into the box
    c->hx.resize(n);
    c->hy.resize(n);
    c->hz.resize(n);
    c->hq.assign(qv, qv + n);
    double qsum = 0, qabs = 0;
    for (int64_t i = 0; i < n; ++i) {
        double p3[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(p3[d])) return fail(c, FMMKMC_EDOMAIN, "non-finite position");
            if (c->bc == FMMKMC_PERIODIC)
                p3[d] = wrap_coord(p3[d], c->a);
            else if (!(p3[d] >= 0.0 && p3[d] < c->a))
                return fail(c, FMMKMC_EDOMAIN, "charge " + std::to_string(i) + " outside the box");
        }
        if (!std::isfinite(qv[i])) return fail(c, FMMKMC_EINVAL, "non-finite charge");
        c->hx[i] = p3[0];
        c->hy[i] = p3[1];
        c->hz[i] = p3[2];
        qsum += qv[i];
        qabs += std::fabs(qv[i]);
    }
    if (c->bc == FMMKMC_PERIODIC && std::fabs(qsum) > 1e-12 * std::max(1.0, qabs))
        return fail(c, FMMKMC_EINVAL, "periodic box must be neutral");
    // cells, sites, capacity
    c->hcell.resize(n);
    c->hsite.assign(n, -1);
    std::vector<int32_t> count(c->M, 0);
    for (int64_t i = 0; i < n; ++i) {
        double p3[3] = {c->hx[i], c->hy[i], c->hz[i]};
        int g[3];
        fine_of(c, p3, g);
        c->hcell[i] = (int32_t)cell_id(c->nc, g[0], g[1], g[2]);
        count[c->hcell[i]]++;
    }
    if (c->lat_n > 0) {
        const int64_t ns = (int64_t)c->lat_n * c->lat_n * c->lat_n;
        c->hsite_charge.assign(ns, -1);
        for (int64_t i = 0; i < n; ++i) {
            double p3[3] = {c->hx[i], c->hy[i], c->hz[i]};
            const int64_t s = site_of(c, p3);
            if (s < 0) return fail(c, FMMKMC_EDOMAIN, "charge " + std::to_string(i) + " is not on a lattice site");
            if (c->hsite_charge[s] >= 0) return fail(c, FMMKMC_ECOINCIDENT, "two charges on one site");
            c->hsite_charge[s] = (int32_t)i;
            c->hsite[i] = (int32_t)s;
        }
        // sites per cell along one axis
        std::vector<int> per(c->nc, 0);
        const double w = c->a / c->nc;
        for (int i = 0; i < c->lat_n; ++i) per[fine_coord((i + 0.5) * c->h, w, c->nc)]++;
        const int mx = *std::max_element(per.begin(), per.end());
        c->cap = prm->cell_capacity > 0 ? prm->cell_capacity : mx * mx * mx;
        c->s2 = (c->lat_n == 2 * c->nc);
    } else {
        const int mx = *std::max_element(count.begin(), count.end());
        c->cap = prm->cell_capacity > 0 ? prm->cell_capacity : std::max(8, 4 * mx);
    }
    int mxc = *std::max_element(count.begin(), count.end());
    if (mxc > c->cap) return fail(c, FMMKMC_ECAPACITY, "a fine cell holds more charges than cell_capacity");
    c->hcnt.assign(c->M, 0);
    c->hslots.assign((size_t)c->M * c->cap, -1);
    c->hslot.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t cl = c->hcell[i];
        c->hslot[i] = c->hcnt[cl];
        c->hslots[(size_t)cl * c->cap + c->hcnt[cl]] = (int32_t)i;
        c->hcnt[cl]++;
    }
    if (c->lat_n == 0) {
        // exact coincidences within a cell
        for (int64_t cl = 0; cl < c->M; ++cl)
            for (int a = 0; a < c->hcnt[cl]; ++a)
                for (int b = a + 1; b < c->hcnt[cl]; ++b) {
                    const int i = c->hslots[cl * c->cap + a], j = c->hslots[cl * c->cap + b];
                    if (c->hx[i] == c->hx[j] && c->hy[i] == c->hy[j] && c->hz[i] == c->hz[j])
                        return fail(c, FMMKMC_ECOINCIDENT, "two charges at one point");
                }
    }
    // device state
    const hipStream_t s = c->stream;
    c->x = dalloc<double>(n);
    c->y = dalloc<double>(n);
    c->z = dalloc<double>(n);
    c->q = dalloc<double>(n);
    upload(c->x, c->hx.data(), n, s);
    upload(c->y, c->hy.data(), n, s);
    upload(c->z, c->hz.data(), n, s);
    upload(c->q, c->hq.data(), n, s);
    c->cell = dalloc<int32_t>(n);
    c->slot = dalloc<int32_t>(n);
    c->site = dalloc<int32_t>(n);
    upload(c->cell, c->hcell.data(), n, s);
    upload(c->slot, c->hslot.data(), n, s);
    upload(c->site, c->hsite.data(), n, s);
    c->cell_cnt = dalloc<int32_t>(c->M);
    c->cell_slots = dalloc<int32_t>((size_t)c->M * c->cap);
    upload(c->cell_cnt, c->hcnt.data(), c->M, s);
    upload(c->cell_slots, c->hslots.data(), (size_t)c->M * c->cap, s);
    {
        std::vector<int64_t> io(n);
        for (int64_t i = 0; i < n; ++i) io[i] = i;
        c->iota = dalloc<int64_t>(n);
        upload(c->iota, io.data(), n, s);
        HIPCHK(hipStreamSynchronize(s));
    }
    c->phi_lv.assign(c->L + 1, nullptr);
    c->psi_lv.assign(c->L + 1, nullptr);
    for (int l = 1; l <= c->L; ++l) {
        const int64_t ml = (int64_t)1 << (3 * (l - 1));
        c->phi_lv[l] = dalloc<double>((size_t)ml * c->nt);
        c->psi_lv[l] = dalloc<double>((size_t)ml * c->nt);
        HIPCHK(hipMemsetAsync(c->psi_lv[l], 0, sizeof(double) * ml * c->nt, s));
    }
    c->d_phi_ptrs = dalloc<double *>(c->L + 1);
    upload(c->d_phi_ptrs, c->phi_lv.data(), c->L + 1, s);
    c->d_psi_ptrs = dalloc<double *>(c->L + 1);
    upload(c->d_psi_ptrs, c->psi_lv.data(), c->L + 1, s);
    if (c->prec == FMMKMC_MIXED) c->psi32 = dalloc<float>((size_t)c->M * c->nt);
    if (c->lat_n > 0) {
        const int64_t ns = (int64_t)c->lat_n * c->lat_n * c->lat_n;
        {
            std::vector<int32_t> sc(ns, -1), ord, pk(n);
            std::vector<double> qr(n);
            for (int64_t i = 0; i < n; ++i) sc[site_order(c, c->hsite[i])] = (int32_t)i;
            ord.reserve(n);
            for (int64_t so = 0; so < ns; ++so)
                if (sc[so] >= 0) ord.push_back(sc[so]);
            c->hrank.assign(n, 0);
            for (int64_t r = 0; r < n; ++r) {
                const int32_t i = ord[r];
                c->hrank[i] = (int32_t)r;
                pk[r] = pack_ijk(c, c->hsite[i]);
                qr[r] = c->hq[i];
            }
            c->site_charge = dalloc<int32_t>(ns);
            upload(c->site_charge, sc.data(), ns, s);
            std::vector<int32_t> sr(ns, -1);
            for (int64_t so = 0; so < ns; ++so)
                if (sc[so] >= 0) sr[so] = c->hrank[sc[so]];
            c->site_rank = dalloc<int32_t>(ns);
            upload(c->site_rank, sr.data(), ns, s);
            c->phi_r = dalloc<double>(n);
            c->order = dalloc<int32_t>(n);
            upload(c->order, ord.data(), n, s);
            c->rank_of = dalloc<int32_t>(n);
            upload(c->rank_of, c->hrank.data(), n, s);
            c->ijk_r = dalloc<int32_t>(n);
            upload(c->ijk_r, pk.data(), n, s);
            c->q_r = dalloc<double>(n);
            upload(c->q_r, qr.data(), n, s);
            HIPCHK(hipStreamSynchronize(s));
        }
        c->phisite = dalloc<double>(ns);
        // per-level mode: the coarser levels' potential per site (none when only the fine level has an
        // interaction list)
        const int lstart = c->bc == FMMKMC_PERIODIC ? 2 : 3;
        if (c->per_level && c->L - 1 >= lstart) c->phicoarse = dalloc<double>(ns * (c->s2 ? c->L - lstart : 1));
        {
            // charge per site in site order (0 on a vacant site)
            std::vector<double> qs(ns, 0.0);
            std::vector<float> qs32(ns, 0.0f);
            bool q32exact = true;
            for (int64_t i = 0; i < n; ++i) {
                const int64_t so = site_order(c, c->hsite[i]);
                qs[so] = c->hq[i];
                qs32[so] = (float)c->hq[i];
                q32exact = q32exact && (double)qs32[so] == c->hq[i];
            }
            // per axis, the first and last lattice plane of every fine cell (the
            // cell of a site is the cell of its position, as for any point):
            // first = planes in lower cells, last = planes in this and lower
            // cells - 1, so a cell holding no plane has an empty range at the
            // right place and runs of consecutive cells are [first, last]
            std::vector<int32_t> rng(2 * (size_t)c->nc, 0), per(c->nc, 0);
            const double w = c->a / c->nc, h = lattice_h(c);
            for (int i = 0; i < c->lat_n; ++i) ++per[fine_coord((i + 0.5) * h, w, c->nc)];
            int below = 0;
            for (int cc = 0; cc < c->nc; ++cc) {
                rng[2 * cc] = below;
                below += per[cc];
                rng[2 * cc + 1] = below - 1;
            }
            c->cell_rng = dalloc<int32_t>(rng.size());
            upload(c->cell_rng, rng.data(), rng.size(), s);
            // widest run of planes in three consecutive cells: bounds every offset of a near field
            int span = 0;
            for (int cc = 0; cc < c->nc; ++cc) {
                int planes = 0;
                for (int d = -1; d <= 1; ++d) {
                    int a2 = cc + d;
                    if (a2 < 0 || a2 >= c->nc) {
                        if (c->bc != FMMKMC_PERIODIC) continue;
                        a2 = (a2 + c->nc) % c->nc;
                    }
                    planes += per[a2];
                }
                span = std::max(span, planes);
            }
            c->near_tab_ok = 3 * (span - 1) * (span - 1) < kInvTab ? 1 : 0;
            c->qsite = dalloc<double>(ns);
            upload(c->qsite, qs.data(), ns, s);
            // FP32 site charges: the mixed near field, and the FP64 one of general
            // lattices when no charge is rounded by FP32
            if (c->prec == FMMKMC_MIXED || (!c->s2 && q32exact)) {
                c->qsite32 = dalloc<float>(ns);
                upload(c->qsite32, qs32.data(), ns, s);
            }
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    c->flags = dalloc<int32_t>(4);
    c->red = dalloc<double>(4096);
    c->acc_buf = dalloc<double>(32);
    build_operators(c);
    if (c->bc == FMMKMC_PERIODIC) build_far(c);
    HIPCHK(hipStreamSynchronize(s));
    return FMMKMC_OK;
}

// energy partial sums of 1/2 q_i phi_i per block
__global__ void k_energy_partials(int64_t n, const double *__restrict__ q, const double *__restrict__ phi,
                                  double *__restrict__ partials)
{
    __shared__ double sm[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += 0.5 * q[i] * phi[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

__global__ void k_interleave(int64_t n, const double *x, const double *y, const double *z, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[3 * i] = x[i];
    out[3 * i + 1] = y[i];
    out[3 * i + 2] = z[i];
}

// CSR of a generic proposal call checked on the device: flag 8 when offs[0] != 0 or
// offs decreases, flag 16 when a charge index is out of range
__global__ void k_check_csr(int64_t G, const int64_t *__restrict__ idx, const int64_t *__restrict__ offs, int64_t N,
                            int32_t *__restrict__ flags)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0 && offs[0] != 0) atomicOr(flags, 8);
    if (g >= G) return;
    if (offs[g + 1] < offs[g]) atomicOr(flags, 8);
    if (idx[g] < 0 || idx[g] >= N) atomicOr(flags, 16);
}

int read_flags(fmmkmc_ctx *c, int32_t *out)
{
    HIPCHK(hipMemcpyAsync(out, c->flags, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

void clear_flags(fmmkmc_ctx *c) { HIPCHK(hipMemsetAsync(c->flags, 0, sizeof(int32_t) * 4, c->stream)); }

}  // namespace

namespace fmmkmc {

Geo make_geo(const fmmkmc_ctx *c)
{
    Geo g;
    g.a = c->a;
    g.w = c->a / c->nc;
    g.h = c->h;
    g.nc = c->nc;
    g.n = c->lat_n;
    g.periodic = c->bc == FMMKMC_PERIODIC ? 1 : 0;
    g.cap = c->cap;
    g.tab_ok = c->near_tab_ok;
    g.self_exact = c->self_exact;
    g.per_level = c->per_level;
    g.L = c->L;
    g.lstart = c->bc == FMMKMC_PERIODIC ? 2 : 3;
    g.q32 = c->qsite32 ? 1 : 0;
    g.ncoarse = c->phicoarse ? (c->s2 ? c->L - g.lstart : 1) : 0;
    for (int k = 0; k < 3; ++k) g.field[k] = c->field[k];
    return g;
}

void Profiler::resolve()
{
    for (auto &pd : pending) {
        (void)hipEventSynchronize(pd.b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, pd.a, pd.b);
        auto &t = total[pd.name];
        t.first += ms;
        t.second += 1;
        (void)hipEventDestroy(pd.a);
        (void)hipEventDestroy(pd.b);
    }
    pending.clear();
}

}  // namespace fmmkmc

extern "C" {

int fmmkmc_create(const fmmkmc_params *prm, int64_t n, const double *xyz, const double *q, fmmkmc_ctx **out)
{
    if (!out) return FMMKMC_EINVAL;
    *out = nullptr;
    fmmkmc_ctx *c = new (std::nothrow) fmmkmc_ctx();
    if (!c) return FMMKMC_ENOMEM;
    int rc;
    try {
        rc = create_impl(prm, n, xyz, q, c);
    } catch (const HipError &e) {
        rc = fail(c, FMMKMC_EHIP, e.what);
    } catch (const std::bad_alloc &) {
        rc = fail(c, FMMKMC_ENOMEM, "device or host allocation failed");
    }
    if (rc != FMMKMC_OK) {
        create_error() = c->err;
        release(c);
        delete c;
        return rc;
    }
    *out = c;
    return FMMKMC_OK;
}

int fmmkmc_initialise(fmmkmc_ctx *c, double *U_out)
{
    if (!c) return FMMKMC_EINVAL;
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        const Geo g = make_geo(c);
        launch_p2m(c, g);
        launch_upward(c);
        launch_downward(c);
        if (c->prec == FMMKMC_MIXED) launch_shadow(c);
        if (c->bc == FMMKMC_PERIODIC) launch_far_refresh(c);
        double *phi = (double *)work_buffer(c, sizeof(double) * c->N);
        // the total energy is always evaluated from the FP64 expansions
        launch_point_phi(c, g, c->N, nullptr, c->iota, c->iota, c->bc == FMMKMC_PERIODIC ? 1 : 0, phi,
                         "point_phi_energy", true);
        const int nb = 1024;
        launch(c, "energy_partials", k_energy_partials, dim3(nb), dim3(256), c->N, c->q, phi, c->red);
        std::vector<double> part(nb);
        HIPCHK(hipMemcpyAsync(part.data(), c->red, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double U = 0.0;
        for (double v : part) U += v;
        c->U = U;
        c->initialised = true;
        c->F_offsets.clear();
        if (U_out) *U_out = U;
        return FMMKMC_OK;
    })
}

int fmmkmc_propose(fmmkmc_ctx *c, int64_t n_groups, const int64_t *idx, const int64_t *offs, const double *targets,
                   double *dU)
{
    if (!c) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "propose before initialise");
    if (n_groups < 0 || (n_groups > 0 && (!idx || !offs || !targets || !dU)))
        return fail(c, FMMKMC_EINVAL, "bad propose arguments");
    if (n_groups == 0) return FMMKMC_OK;
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        // the CSR drives device writes: check it on the host first
        std::vector<int64_t> hoffs(n_groups + 1);
        HIPCHK(hipMemcpyAsync(hoffs.data(), offs, sizeof(int64_t) * (n_groups + 1), hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (hoffs[0] != 0) return fail(c, FMMKMC_EINVAL, "offs[0] must be 0");
        for (int64_t g2 = 0; g2 < n_groups; ++g2)
            if (hoffs[g2 + 1] < hoffs[g2]) return fail(c, FMMKMC_EINVAL, "offs must be non-decreasing");
        const int64_t S = hoffs[n_groups];
        if (S == 0) return FMMKMC_OK;
        std::vector<int64_t> hidx(n_groups);
        HIPCHK(hipMemcpyAsync(hidx.data(), idx, sizeof(int64_t) * n_groups, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int64_t v : hidx)
            if (v < 0 || v >= c->N) return fail(c, FMMKMC_EINVAL, "charge index out of range");
        const size_t bytes = sizeof(double) * 8 * S + sizeof(int64_t) * S;
        double *work = (double *)work_buffer(c, bytes);
        int64_t *charge = (int64_t *)(work + 8 * S);
        clear_flags(c);
        const Geo g = make_geo(c);
        launch_expand_groups(c, n_groups, idx, offs, charge);
        launch_generic(c, g, S, targets, charge, dU, work);
        int32_t fl = 0;
        read_flags(c, &fl);
        if (fl & 1) return fail(c, FMMKMC_EDOMAIN, "a target lies outside the box (NaN written)");
        if (fl & 2) return fail(c, FMMKMC_ECOINCIDENT, "a target coincides with a charge (NaN written)");
        return FMMKMC_OK;
    })
}

int fmmkmc_propose_noalloc(fmmkmc_ctx *c, int64_t n_groups, const int64_t *idx, const int64_t *offs,
                           const double *targets, double *dU)
{
    if (!c) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "propose before initialise");
    if (n_groups < 0 || (n_groups > 0 && (!idx || !offs || !targets || !dU)))
        return fail(c, FMMKMC_EINVAL, "bad propose arguments");
    if (n_groups == 0) return FMMKMC_OK;
    if (c->device < 0 || c->device >= kMaxScratchDevices)
        return fail(c, FMMKMC_EINVAL, "device ordinal beyond the work-array table");
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        void *base = device_scratch(c->device);  // resolved at context creation: a table lookup
        clear_flags(c);
        launch(c, "check_csr", k_check_csr, dim3((unsigned)((n_groups + 255) / 256)), dim3(256), n_groups, idx, offs,
               c->N, c->flags);
        int32_t fl = 0;
        int64_t S = 0;
        HIPCHK(hipMemcpyAsync(&fl, c->flags, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(&S, offs + n_groups, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (fl & 8) return fail(c, FMMKMC_EINVAL, "offs[0] must be 0 and offs non-decreasing");
        if (fl & 16) return fail(c, FMMKMC_EINVAL, "charge index out of range");
        if (S == 0) return FMMKMC_OK;
        if (S > kNoAllocSlots) return fail(c, FMMKMC_EINVAL, "at most 262144 targets per allocation-free call");
        // the same work layout as fmmkmc_propose: 8 doubles per slot, then the charge index per slot
        double *work = (double *)base;
        int64_t *charge = (int64_t *)(work + 8 * S);
        clear_flags(c);
        const Geo g = make_geo(c);
        launch_expand_groups(c, n_groups, idx, offs, charge);
        launch_generic(c, g, S, targets, charge, dU, work);
        read_flags(c, &fl);
        if (fl & 1) return fail(c, FMMKMC_EDOMAIN, "a target lies outside the box (NaN written)");
        if (fl & 2) return fail(c, FMMKMC_ECOINCIDENT, "a target coincides with a charge (NaN written)");
        return FMMKMC_OK;
    })
}

int fmmkmc_propose_dats(fmmkmc_ctx *c, int K, const int32_t *C, int n_types, const int32_t *T, const double *R,
                        const uint8_t *Mk, double *U)
{
    if (!c) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "propose before initialise");
    if (K < 0 || n_types < 1 || !C || !T || !R || !Mk || !U) return fail(c, FMMKMC_EINVAL, "bad dats arguments");
    for (int t = 0; t < n_types; ++t)
        if (C[t] < 0 || C[t] > K) return fail(c, FMMKMC_EINVAL, "C[t] must be in 0..K");
    if (K == 0) return FMMKMC_OK;
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        const int64_t S = c->N * K;
        const size_t bytes = sizeof(double) * 8 * S + sizeof(int64_t) * S + sizeof(int32_t) * (S + n_types);
        double *work = (double *)work_buffer(c, bytes);
        int64_t *charge = (int64_t *)(work + 8 * S);
        int32_t *use = (int32_t *)(charge + S);
        int32_t *dC = use + S;
        upload(dC, C, n_types, c->stream);
        clear_flags(c);
        const Geo g = make_geo(c);
        launch_dats_select(c, c->N, K, dC, n_types, T, Mk, use);
        // every slot (i, k) is a proposal of charge i; unused slots come out as NaN
        launch_div_index(c, S, K, charge);
        launch_generic(c, g, S, R, charge, U, work, use);
        int32_t fl = 0;
        read_flags(c, &fl);
        if (fl & 4) return fail(c, FMMKMC_EINVAL, "a particle type is out of range");
        if (fl & 1) return fail(c, FMMKMC_EDOMAIN, "an allowed target lies outside the box (NaN written)");
        if (fl & 2) return fail(c, FMMKMC_ECOINCIDENT, "an allowed target coincides with a charge (NaN written)");
        return FMMKMC_OK;
    })
}

int fmmkmc_propose_lattice(fmmkmc_ctx *c, int K, const int32_t *offsets, double *dU, uint8_t *mask)
{
    if (!c) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "propose before initialise");
    if (c->lat_n <= 0) return fail(c, FMMKMC_ESTATE, "context was not created in lattice mode");
    if (K < 1 || K > kMaxHops || !offsets || !dU) return fail(c, FMMKMC_EINVAL, "need 1 <= K <= 64 and dU");
    if (c->N * (int64_t)K >= ((int64_t)1 << 32)) return fail(c, FMMKMC_EINVAL, "N * K must be < 2^32");
    for (int k = 0; k < 3 * K; ++k)
        if (offsets[k] < -1 || offsets[k] > 1) return fail(c, FMMKMC_EINVAL, "hop offsets must be in -1..1");
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        const Geo g = make_geo(c);
        std::vector<int32_t> off(offsets, offsets + 3 * K);
        if (off != c->F_offsets) {
            dfree(c->d_offsets);
            c->d_offsets = dalloc<int32_t>(3 * K);
            upload(c->d_offsets, off.data(), 3 * K, c->stream);
            c->d_offsets_K = K;
            if (c->bc == FMMKMC_PERIODIC && c->self_exact) {
                dfree(c->Fhop);
                c->Fhop = dalloc<double>(K);
                launch_self_hops(c, K);
            } else if (c->bc == FMMKMC_PERIODIC) {
                if (!c->far.sigma) {
                    const int64_t ns = (int64_t)c->lat_n * c->lat_n * c->lat_n;
                    c->far.sigma = dalloc<double>(ns);
                    launch_sigma(c, g);
                }
                dfree(c->F);
                c->F = dalloc<double>((size_t)c->N * K);
                if (!c->frow_w) c->frow_w = dalloc<double>(c->nt);
                launch_f_rows(c, g, c->N, K, 0);
            }
            c->F_offsets = off;
        }
        launch_coarse_sites(c, g);  // per-level mode: the levels above the fine one
        launch_site_phi(c, g);
        launch_slot_lattice(c, g, K, dU, mask);
        return FMMKMC_OK;
    })
}

int fmmkmc_accept(fmmkmc_ctx *c, int64_t i, const double new_xyz[3], double *dU_out)
{
    if (!c) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "accept before initialise");
    if (i < 0 || i >= c->N || !new_xyz) return fail(c, FMMKMC_EINVAL, "bad charge index or position");
    if (c->dev_ahead) {
        API_GUARD(c, { refresh_mirrors(c); })
    }
    double np[3];
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(new_xyz[d])) return fail(c, FMMKMC_EDOMAIN, "non-finite position");
        if (c->bc == FMMKMC_PERIODIC)
            np[d] = wrap_coord(new_xyz[d], c->a);
        else if (!(new_xyz[d] >= 0.0 && new_xyz[d] < c->a))
            return fail(c, FMMKMC_EDOMAIN, "new position outside the box");
        else
            np[d] = new_xyz[d];
    }
    const double op[3] = {c->hx[i], c->hy[i], c->hz[i]};
    int og[3], ng[3];
    fine_of(c, op, og);
    fine_of(c, np, ng);
    const int64_t old_cell = c->hcell[i], new_cell = cell_id(c->nc, ng[0], ng[1], ng[2]);
    int64_t old_site = -1, new_site = -1;
    if (c->lat_n > 0) {
        old_site = c->hsite[i];
        new_site = site_of(c, np);
        if (new_site < 0) return fail(c, FMMKMC_EDOMAIN, "new position is not a lattice site");
        if (c->hsite_charge[new_site] >= 0) return fail(c, FMMKMC_ECOINCIDENT, "target site is occupied");
    } else {
        for (int k = 0; k < c->hcnt[new_cell]; ++k) {
            const int j = c->hslots[(size_t)new_cell * c->cap + k];
            if (c->hx[j] == np[0] && c->hy[j] == np[1] && c->hz[j] == np[2])
                return fail(c, FMMKMC_ECOINCIDENT, "target coincides with a charge");
        }
    }
    if (new_cell != old_cell && c->hcnt[new_cell] >= c->cap)
        return fail(c, FMMKMC_ECAPACITY, "target cell is full");
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        const Geo g = make_geo(c);
        // C1: dU of the move (footnote to Sec. 3.1) as partial sums, read back
        // after the commit kernels are queued behind it (one synchronisation per accept)
        double *dUd = c->acc_buf;
        // the part that reads the fine-level expansions, before the sweep
        launch_move_dU(c, g, i, np, dUd, c->stream, 0, 1);
        // The work beside the sweep goes to the side stream, after every earlier
        // proposal (they read the old state): the rest of the move's dU (cell
        // lists and far-field tables, read before the bookkeeping and the
        // far-field refresh change them), the moved charge's row of the lattice
        // proposal table (it depends only on the new site), the multipole path,
        // the bookkeeping and the far-field refresh.  None of it touches the
        // fine-level expansions or what the sweep reads.
        const bool need_row = c->bc == FMMKMC_PERIODIC && !c->self_exact && c->F && !c->F_offsets.empty();
        const int Krow = (int)c->F_offsets.size() / 3;
        HIPCHK(hipEventRecord(c->ev_fork, c->stream));
        HIPCHK(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
        launch_move_dU(c, g, i, np, dUd, c->aux, 1, kMoveParts - 1);
        if (need_row) launch_f_row1(c, g, Krow, c->hrank[i], new_site, c->aux);
        // C2 + C3
        CommitArgs a;
        a.i = i;
        std::memcpy(a.old_pos, op, sizeof(op));
        std::memcpy(a.new_pos, np, sizeof(np));
        a.q = c->hq[i];
        std::memcpy(a.old_g, og, sizeof(og));
        std::memcpy(a.new_g, ng, sizeof(ng));
        a.old_cell = old_cell;
        a.new_cell = new_cell;
        a.old_slot = c->hslot[i];
        a.moved_j = -1;
        a.new_slot = c->hslot[i];
        a.old_cnt = c->hcnt[old_cell];
        a.new_cnt = c->hcnt[new_cell];
        if (new_cell != old_cell) {
            const int last = c->hcnt[old_cell] - 1;
            const int jlast = c->hslots[(size_t)old_cell * c->cap + last];
            a.moved_j = (jlast != i) ? jlast : -1;
            a.old_cnt = last;
            a.new_slot = c->hcnt[new_cell];
            a.new_cnt = c->hcnt[new_cell] + 1;
        }
        a.old_site = old_site;
        a.new_site = new_site;
        a.old_sord = a.new_sord = -1;
        a.new_ijk = 0;
        if (c->lat_n > 0) {
            a.old_sord = site_order(c, old_site);
            a.new_sord = site_order(c, new_site);
            a.new_ijk = pack_ijk(c, new_site);
            a.rank = c->hrank[i];
        }
        launch_commit(c, g, a, c->aux);
        if (c->bc == FMMKMC_PERIODIC) launch_far_refresh(c, c->aux);
        HIPCHK(hipEventRecord(c->ev_join, c->aux));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
        // host mirrors
        c->hx[i] = np[0];
        c->hy[i] = np[1];
        c->hz[i] = np[2];
        if (new_cell != old_cell) {
            if (a.moved_j >= 0) {
                c->hslots[(size_t)old_cell * c->cap + a.old_slot] = a.moved_j;
                c->hslot[a.moved_j] = a.old_slot;
            }
            c->hslots[(size_t)old_cell * c->cap + a.old_cnt] = -1;
            c->hcnt[old_cell] = a.old_cnt;
            c->hslots[(size_t)new_cell * c->cap + a.new_slot] = (int32_t)i;
            c->hcnt[new_cell] = a.new_cnt;
            c->hcell[i] = (int32_t)new_cell;
            c->hslot[i] = a.new_slot;
        }
        if (c->lat_n > 0) {
            c->hsite_charge[old_site] = -1;
            c->hsite_charge[new_site] = (int32_t)i;
            c->hsite[i] = (int32_t)new_site;
        }
        double parts[kMoveParts];
        HIPCHK(hipMemcpyAsync(parts, dUd, sizeof(parts), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double dUh = 0;
        for (int k = 0; k < kMoveParts; ++k) dUh += parts[k];
        if (dU_out) *dU_out = dUh;
        c->U += dUh;
        return FMMKMC_OK;
    })
}

int fmmkmc_set_field(fmmkmc_ctx *c, const double E[3])
{
    if (!c || !E) return FMMKMC_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(E[k])) return fail(c, FMMKMC_EINVAL, "field components must be finite");
    for (int k = 0; k < 3; ++k) c->field[k] = E[k];
    return FMMKMC_OK;
}

int fmmkmc_energy(fmmkmc_ctx *c, double *U)
{
    if (!c || !U) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "energy before initialise");
    *U = c->U;
    return FMMKMC_OK;
}

int fmmkmc_positions(fmmkmc_ctx *c, double *xyz)
{
    if (!c || !xyz) return FMMKMC_EINVAL;
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        launch(c, "interleave", k_interleave, dim3((unsigned)((c->N + 255) / 256)), dim3(256), c->N, c->x, c->y,
               c->z, xyz);
        HIPCHK(hipStreamSynchronize(c->stream));
        return FMMKMC_OK;
    })
}

int fmmkmc_potential(fmmkmc_ctx *c, int64_t m, const double *xyz, const int64_t *exclude, double *out)
{
    if (!c || m < 0 || (m > 0 && (!xyz || !out))) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "potential before initialise");
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        launch_point_phi(c, make_geo(c), m, xyz, nullptr, exclude, c->bc == FMMKMC_PERIODIC ? 1 : 0, out,
                         "point_phi");
        HIPCHK(hipStreamSynchronize(c->stream));
        return FMMKMC_OK;
    })
}

int fmmkmc_multipole(fmmkmc_ctx *c, int level, int64_t cell, double *out)
{
    if (!c || !out) return FMMKMC_EINVAL;
    if (!c->initialised) return fail(c, FMMKMC_ESTATE, "multipole before initialise");
    if (level < 1 || level > c->L) return fail(c, FMMKMC_EINVAL, "level must be in 1..L");
    const int64_t side = (int64_t)1 << (level - 1), cells = side * side * side;
    if (cell < 0 || cell >= cells) return fail(c, FMMKMC_EINVAL, "cell index out of range for the level");
    API_GUARD(c, {
        HIPCHK(hipSetDevice(c->device));
        // coefficient-major storage: coefficient k of the cell sits at [k * cells + cell]
        HIPCHK(hipMemcpy2DAsync(out, sizeof(double), c->phi_lv[level] + cell, sizeof(double) * cells, sizeof(double),
                                (size_t)c->nt, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return FMMKMC_OK;
    })
}

int fmmkmc_set_profiling(fmmkmc_ctx *c, int on)
{
    if (!c) return FMMKMC_EINVAL;
    API_GUARD(c, {
        c->prof.resolve();
        c->prof.total.clear();
        c->prof.on = on != 0;
        return FMMKMC_OK;
    })
}

int fmmkmc_kernel_time(fmmkmc_ctx *c, const char *name, double *ms, int64_t *launches)
{
    if (!c || !name) return FMMKMC_EINVAL;
    c->prof.resolve();
    auto it = c->prof.total.find(name);
    if (ms) *ms = it == c->prof.total.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == c->prof.total.end() ? 0 : it->second.second;
    return FMMKMC_OK;
}

const char *fmmkmc_last_error(fmmkmc_ctx *c)
{
    if (!c) return create_error().c_str();
    return c->err.c_str();
}

int fmmkmc_destroy(fmmkmc_ctx *c)
{
    if (!c) return FMMKMC_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
    return FMMKMC_OK;
}

}  // extern "C"
