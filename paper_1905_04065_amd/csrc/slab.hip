// Charges between two grounded plates (Sec. 2.2.2, "Dirichlet"): the potential
// vanishes on the planes z = 0 and z = c, and the system is periodic with
// period a = 2c in x and y.  As the paper describes, the physical slab
// [0, a) x [0, a) x [0, c) is extended by its first mirror image (charge -q at
// (x, y, a - z) for every charge q at (x, y, z)) and the doubled system is
// treated with the periodic algorithm.  The doubled charge distribution is odd
// under the reflections about z = 0 and z = c, so its periodic (conducting
// boundary) potential vanishes on both planes.  A uniform external field E_z
// along z (the applied voltage of Sec. 6.3) adds -E_z q z per charge.
//
// Energies: the doubled system holds every physical interaction twice (each
// charge and its mirror see the same potential with opposite sign), so the
// physical energy is half the periodic energy of the doubled system, plus the
// field term.  A hop of charge i is a joint move of i and its mirror m:
//   dU_pair = dU_i + dU_m + q_i q_m [G(r_i' - r_m') - G(r_i' - r_m) - G(r_i - r_m') + G(r_i - r_m)],
// with dU_i and dU_m the single-move values of the periodic path (each taken
// with the partner at its old place) and G the periodic pair potential; the
// bracket corrects the partner term.  For lattice hops it depends only on the
// height of the site and the hop, and it is tabulated once with an Ewald sum
// (conducting boundary).  The physical dU is dU_pair / 2 - E_z q dz.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fmmkmc.h"
#include "ewald.hpp"
#include "hostutil.hpp"

using namespace fmmkmc;

namespace {

// bracket of the pair move for a charge on layer zi (z = (zi + 1/2) h) and hop
// k with offsets (dx, dy, dz): G(d1) - 2 G(d2) + G(d4) (the two mixed terms are
// equal by the lattice's reflection symmetry in x and y); 0 where the hop leaves
// the slab (such slots are masked)
__global__ void k_slab_cross(int half, int K, const int32_t *__restrict__ offs, double h, double a,
                             double *__restrict__ cross)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= half * K) return;
    const int zi = e / K, k = e - zi * K;
    const int dx = offs[3 * k], dy = offs[3 * k + 1], dz = offs[3 * k + 2];
    const int tz = zi + dz;
    if (tz < 0 || tz >= half) {
        cross[e] = 0.0;
        return;
    }
    const double z = (zi + 0.5) * h, zt = (tz + 0.5) * h;
    const double g1 = periodic_g(0.0, 0.0, 2.0 * zt - a, a);                 // r_i' - r_m'
    const double g2 = periodic_g(dx * h, dy * h, z + zt - a, a);             // r_i' - r_m
    const double g4 = periodic_g(0.0, 0.0, 2.0 * z - a, a);                  // r_i - r_m
    cross[e] = g1 - 2.0 * g2 + g4;
}

// physical dU and mask of every (charge, hop) slot from the doubled system's
// proposal pass: charge i's slot k with its mirror's (N + i) slot mk[k]
__global__ void k_slab_pairs(int64_t N, int K, int half, double h, double ez, const double *__restrict__ dU2,
                             const uint8_t *__restrict__ mask2, const double *__restrict__ z,
                             const double *__restrict__ q, const int32_t *__restrict__ offs,
                             const int32_t *__restrict__ mk, const double *__restrict__ cross,
                             double *__restrict__ dU, uint8_t *__restrict__ mask)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * K) return;
    const int64_t i = e / K;
    const int k = (int)(e - i * K);
    const int zi = (int)floor(z[i] / h);
    const int dz = offs[3 * k + 2];
    const int tz = zi + dz;
    const int64_t em = (N + i) * K + mk[k];
    const bool valid = tz >= 0 && tz < half && mask2[e] && mask2[em];
    const double qi = q[i];
    // q_i q_m = -q_i^2 for the mirror
    const double v = valid ? 0.5 * (dU2[e] + dU2[em] - qi * qi * cross[(int64_t)zi * K + k]) - ez * qi * dz * h
                           : __builtin_nan("");
    dU[e] = v;
    if (mask) mask[e] = valid ? 1 : 0;
}

}  // namespace

struct fmmkmc_slab {
    fmmkmc_ctx *ctx = nullptr;  // the doubled periodic system: charges 0..N-1 physical, N..2N-1 mirrors
    int64_t N = 0;
    int n = 0, half = 0;
    double a = 0, h = 0, ez = 0;
    double U = 0;
    bool initialised = false;
    std::string err;
    // hop table of the current offsets
    std::vector<int32_t> offsets;
    int32_t *d_offs = nullptr, *d_mk = nullptr;
    double *cross = nullptr;
    double *dU2 = nullptr;
    uint8_t *mask2 = nullptr;
    double *pos2 = nullptr;
};

namespace {

int sfail(fmmkmc_slab *s, int code, const std::string &msg)
{
    if (s) s->err = msg;
    return code;
}

// pass a status of the inner context on, with its message
int inner(fmmkmc_slab *s, int rc)
{
    if (rc != FMMKMC_OK) s->err = fmmkmc_last_error(s->ctx);
    return rc;
}

#define SLAB_GUARD(s, ...)                                                       \
    try {                                                                        \
        __VA_ARGS__                                                              \
    } catch (const HipError &e) {                                                \
        return sfail(s, FMMKMC_EHIP, e.what);                                    \
    } catch (const std::bad_alloc &) {                                           \
        return sfail(s, FMMKMC_ENOMEM, "device or host allocation failed");      \
    }

void release_slab(fmmkmc_slab *s)
{
    dfree(s->d_offs);
    dfree(s->d_mk);
    dfree(s->cross);
    dfree(s->dU2);
    dfree(s->mask2);
    dfree(s->pos2);
    if (s->ctx) fmmkmc_destroy(s->ctx);
    s->ctx = nullptr;
}

// field energy of the physical charges: -E_z sum q z
double field_energy(const fmmkmc_slab *s)
{
    double u = 0.0;
    for (int64_t i = 0; i < s->N; ++i) u += s->ctx->hq[i] * s->ctx->hz[i];
    return -s->ez * u;
}

}  // namespace

extern "C" {

int fmmkmc_slab_create(const fmmkmc_params *prm, int64_t n, const double *xyz, const double *q, double ez,
                       fmmkmc_slab **out)
{
    if (!out) return FMMKMC_EINVAL;
    *out = nullptr;
    auto err = [](const char *m) {
        create_error() = m;
        return FMMKMC_EINVAL;
    };
    if (!prm || !xyz || !q) return err("null argument");
    if (prm->lattice_n <= 0 || prm->lattice_n % 2) return err("a slab needs lattice mode with an even lattice_n");
    if (!std::isfinite(ez)) return err("the field must be finite");
    if (n < 1 || n > ((int64_t)1 << 29)) return err("charge count out of range");
    const double a = prm->a, h = a / prm->lattice_n;
    for (int64_t i = 0; i < n; ++i)
        if (!(xyz[3 * i + 2] >= 0.0 && xyz[3 * i + 2] < 0.5 * a)) {
            create_error() = "every charge must lie in 0 <= z < a/2";
            return FMMKMC_EDOMAIN;
        }
    fmmkmc_slab *s = new (std::nothrow) fmmkmc_slab();
    if (!s) return FMMKMC_ENOMEM;
    std::vector<double> xyz2(6 * n), q2(2 * n);
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) xyz2[3 * i + d] = xyz[3 * i + d];
        xyz2[3 * (n + i)] = xyz[3 * i];
        xyz2[3 * (n + i) + 1] = xyz[3 * i + 1];
        xyz2[3 * (n + i) + 2] = a - xyz[3 * i + 2];
        q2[i] = q[i];
        q2[n + i] = -q[i];
    }
    fmmkmc_params p2 = *prm;
    p2.bc = FMMKMC_PERIODIC;
    const int rc = fmmkmc_create(&p2, 2 * n, xyz2.data(), q2.data(), &s->ctx);
    if (rc != FMMKMC_OK) {
        delete s;
        return rc;  // create_error() holds the inner message
    }
    s->N = n;
    s->n = prm->lattice_n;
    s->half = prm->lattice_n / 2;
    s->a = a;
    s->h = h;
    s->ez = ez;
    *out = s;
    return FMMKMC_OK;
}

int fmmkmc_slab_initialise(fmmkmc_slab *s, double *U_out)
{
    if (!s) return FMMKMC_EINVAL;
    double U2 = 0.0;
    const int rc = fmmkmc_initialise(s->ctx, &U2);
    if (rc != FMMKMC_OK) return inner(s, rc);
    s->U = 0.5 * U2 + field_energy(s);
    s->initialised = true;
    s->offsets.clear();
    if (U_out) *U_out = s->U;
    return FMMKMC_OK;
}

int fmmkmc_slab_propose_lattice(fmmkmc_slab *s, int K, const int32_t *offsets, double *dU, uint8_t *mask)
{
    if (!s) return FMMKMC_EINVAL;
    if (!s->initialised) return sfail(s, FMMKMC_ESTATE, "propose before initialise");
    if (K < 1 || K > kMaxHops || !offsets || !dU) return sfail(s, FMMKMC_EINVAL, "need 1 <= K <= 64 and dU");
    for (int k = 0; k < 3 * K; ++k)
        if (offsets[k] < -1 || offsets[k] > 1) return sfail(s, FMMKMC_EINVAL, "hop offsets must be in -1..1");
    // the mirror of hop (dx, dy, dz) is (dx, dy, -dz): it must be one of the hops
    std::vector<int32_t> mk(K, -1);
    for (int k = 0; k < K; ++k)
        for (int l = 0; l < K; ++l)
            if (offsets[3 * l] == offsets[3 * k] && offsets[3 * l + 1] == offsets[3 * k + 1] &&
                offsets[3 * l + 2] == -offsets[3 * k + 2]) {
                mk[k] = l;
                break;
            }
    for (int k = 0; k < K; ++k)
        if (mk[k] < 0) return sfail(s, FMMKMC_EINVAL, "the hop set must be closed under dz -> -dz");
    fmmkmc_ctx *c = s->ctx;
    SLAB_GUARD(s, {
        HIPCHK(hipSetDevice(c->device));
        const hipStream_t st = c->stream;
        std::vector<int32_t> off(offsets, offsets + 3 * K);
        if (off != s->offsets) {
            dfree(s->d_offs);
            dfree(s->d_mk);
            dfree(s->cross);
            dfree(s->dU2);
            dfree(s->mask2);
            s->d_offs = dalloc<int32_t>(3 * K);
            s->d_mk = dalloc<int32_t>(K);
            s->cross = dalloc<double>((size_t)s->half * K);
            s->dU2 = dalloc<double>((size_t)2 * s->N * K);
            s->mask2 = dalloc<uint8_t>((size_t)2 * s->N * K);
            upload(s->d_offs, off.data(), 3 * K, st);
            upload(s->d_mk, mk.data(), K, st);
            const int tot = s->half * K;
            hipLaunchKernelGGL(k_slab_cross, dim3((tot + 63) / 64), dim3(64), 0, st, s->half, K,
                               (const int32_t *)s->d_offs, s->h, s->a, s->cross);
            HIPCHK(hipGetLastError());
            s->offsets = off;
        }
        const int rc = fmmkmc_propose_lattice(c, K, offsets, s->dU2, s->mask2);
        if (rc != FMMKMC_OK) return inner(s, rc);
        const int64_t S = s->N * K;
        hipLaunchKernelGGL(k_slab_pairs, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st, s->N, K, s->half, s->h,
                           s->ez, (const double *)s->dU2, (const uint8_t *)s->mask2, (const double *)c->z,
                           (const double *)c->q, (const int32_t *)s->d_offs, (const int32_t *)s->d_mk,
                           (const double *)s->cross, dU, mask);
        HIPCHK(hipGetLastError());
        return FMMKMC_OK;
    })
}

int fmmkmc_slab_accept(fmmkmc_slab *s, int64_t i, const double new_xyz[3], double *dU_out)
{
    if (!s) return FMMKMC_EINVAL;
    if (!s->initialised) return sfail(s, FMMKMC_ESTATE, "accept before initialise");
    if (i < 0 || i >= s->N || !new_xyz) return sfail(s, FMMKMC_EINVAL, "bad charge index or position");
    if (!(new_xyz[2] >= 0.0 && new_xyz[2] < 0.5 * s->a))
        return sfail(s, FMMKMC_EDOMAIN, "the new position must lie in 0 <= z < a/2");
    fmmkmc_ctx *c = s->ctx;
    const double z_old = c->hz[i], q = c->hq[i];
    double d1 = 0.0, d2 = 0.0;
    int rc = fmmkmc_accept(c, i, new_xyz, &d1);
    if (rc != FMMKMC_OK) return inner(s, rc);
    const double mirror[3] = {new_xyz[0], new_xyz[1], s->a - new_xyz[2]};
    rc = fmmkmc_accept(c, s->N + i, mirror, &d2);
    if (rc != FMMKMC_OK) {
        // the physical charge has moved but its mirror could not follow: the
        // doubled system no longer describes the slab
        s->initialised = false;
        inner(s, rc);
        s->err = "mirror move failed after the charge moved (state invalid, initialise again): " + s->err;
        return rc;
    }
    const double dU = 0.5 * (d1 + d2) - s->ez * q * (c->hz[i] - z_old);
    s->U += dU;
    if (dU_out) *dU_out = dU;
    return FMMKMC_OK;
}

int fmmkmc_slab_energy(fmmkmc_slab *s, double *U)
{
    if (!s || !U) return FMMKMC_EINVAL;
    if (!s->initialised) return sfail(s, FMMKMC_ESTATE, "energy before initialise");
    *U = s->U;
    return FMMKMC_OK;
}

int fmmkmc_slab_positions(fmmkmc_slab *s, double *xyz)
{
    if (!s || !xyz) return FMMKMC_EINVAL;
    fmmkmc_ctx *c = s->ctx;
    SLAB_GUARD(s, {
        HIPCHK(hipSetDevice(c->device));
        if (!s->pos2) s->pos2 = dalloc<double>((size_t)6 * s->N);
        const int rc = fmmkmc_positions(c, s->pos2);
        if (rc != FMMKMC_OK) return inner(s, rc);
        HIPCHK(hipMemcpyAsync(xyz, s->pos2, sizeof(double) * 3 * s->N, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return FMMKMC_OK;
    })
}

const char *fmmkmc_slab_last_error(fmmkmc_slab *s)
{
    if (!s) return create_error().c_str();
    return s->err.c_str();
}

int fmmkmc_slab_destroy(fmmkmc_slab *s)
{
    if (!s) return FMMKMC_OK;
    if (s->ctx) {
        (void)hipSetDevice(s->ctx->device);
        (void)hipStreamSynchronize(s->ctx->stream);
    }
    release_slab(s);
    delete s;
    return FMMKMC_OK;
}

}  // extern "C"
