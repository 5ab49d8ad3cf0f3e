// The conducting-boundary ("tin-foil") periodic pair potential of a cubic box,
// by an Ewald split, for host and device code.
//
// G(x) = sum_nu erfc(alpha |x + a nu|) / |x + a nu|
//      + (4 pi / V) sum_{k != 0} exp(-k^2 / (4 alpha^2)) / k^2 cos(k . x)
// without its constant term (-pi / (alpha^2 V), which cancels in every
// difference used here).  The offset is first reduced to its nearest image;
// with alpha = 2.44 / a the real-space images beyond |nu_i| <= 2 and the wave
// vectors beyond |n_i| <= 7 are below 1e-17 of the leading terms.
//
// G_self = lim_{x -> 0} (G(x) - 1/|x|): the same sums without the nu = 0 real
// term, minus 2 alpha / sqrt(pi).
//
// A charge displaced by d from where its own periodic copies sit changes its
// interaction with them by G_self - G(d) (times q^2).  In a periodic proposal
// the FMM potential difference q (phi(r') - phi(r)) holds this term for the
// moving charge; Sec. 3.1 removes it with the V_box self sum, the constant
// (6 + 8/sqrt3 + 12/sqrt2)/a and 1/2 dE.R'dK, which together approximate
// q^2 (G_self - G(r' - r)).  The exact self-image option uses this value.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace fmmkmc {

constexpr double kEwaldAlphaA = 2.44;  // alpha * a
constexpr int kEwaldImages = 2;        // real space: |nu_i| <= 2
constexpr int kEwaldWaves = 7;         // reciprocal space: |n_i| <= 7

__host__ __device__ inline double periodic_g_sums(double x, double y, double z, double a, bool skip_origin)
{
    const double alpha = kEwaldAlphaA / a;
    double real = 0.0;
    for (int i = -kEwaldImages; i <= kEwaldImages; ++i)
        for (int j = -kEwaldImages; j <= kEwaldImages; ++j)
            for (int k = -kEwaldImages; k <= kEwaldImages; ++k) {
                if (skip_origin && i == 0 && j == 0 && k == 0) continue;
                const double dx = x + a * i, dy = y + a * j, dz = z + a * k;
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                real += erfc(alpha * r) / r;
            }
    const double V = a * a * a, tk = 2.0 * M_PI / a;
    double recip = 0.0;
    for (int i = -kEwaldWaves; i <= kEwaldWaves; ++i)
        for (int j = -kEwaldWaves; j <= kEwaldWaves; ++j)
            for (int k = -kEwaldWaves; k <= kEwaldWaves; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                const double kx = tk * i, ky = tk * j, kz = tk * k;
                const double k2 = kx * kx + ky * ky + kz * kz;
                recip += exp(-k2 / (4.0 * alpha * alpha)) / k2 * cos(kx * x + ky * y + kz * z);
            }
    return real + 4.0 * M_PI / V * recip;
}

// G(x) for x not on a lattice point of period a
__host__ __device__ inline double periodic_g(double x, double y, double z, double a)
{
    x -= a * rint(x / a);
    y -= a * rint(y / a);
    z -= a * rint(z / a);
    return periodic_g_sums(x, y, z, a, false);
}

// G_self
__host__ __device__ inline double periodic_g_self(double a)
{
    return periodic_g_sums(0.0, 0.0, 0.0, a, true) - 2.0 * (kEwaldAlphaA / a) / sqrt(M_PI);
}

// G_self - G(d): the change of a unit charge's interaction with its own copies
// when it moves by d (d not a lattice vector)
__host__ __device__ inline double periodic_self_change(double a, double dx, double dy, double dz)
{
    return periodic_g_self(a) - periodic_g(dx, dy, dz, a);
}

}  // namespace fmmkmc

namespace fmmkmc {

// One lane's share of G_self - G(d) when `lanes` lanes split its terms (the
// shares add up to periodic_self_change; used by one block of the accept step)
__device__ inline double periodic_self_change_share(double a, double dx, double dy, double dz, int lane, int lanes)
{
    dx -= a * rint(dx / a);
    dy -= a * rint(dy / a);
    dz -= a * rint(dz / a);
    const double alpha = kEwaldAlphaA / a;
    constexpr int ni = 2 * kEwaldImages + 1, nw = 2 * kEwaldWaves + 1;
    double s = 0.0;
    for (int t = lane; t < ni * ni * ni; t += lanes) {
        const int i = t / (ni * ni) - kEwaldImages, j = (t / ni) % ni - kEwaldImages, k = t % ni - kEwaldImages;
        if (i != 0 || j != 0 || k != 0) {
            const double r0 = a * sqrt((double)(i * i + j * j + k * k));
            s += erfc(alpha * r0) / r0;
        }
        const double ex = dx + a * i, ey = dy + a * j, ez = dz + a * k;
        const double r = sqrt(ex * ex + ey * ey + ez * ez);
        s -= erfc(alpha * r) / r;
    }
    const double V = a * a * a, tk = 2.0 * M_PI / a;
    for (int t = lane; t < nw * nw * nw; t += lanes) {
        const int i = t / (nw * nw) - kEwaldWaves, j = (t / nw) % nw - kEwaldWaves, k = t % nw - kEwaldWaves;
        if (i == 0 && j == 0 && k == 0) continue;
        const double kx = tk * i, ky = tk * j, kz = tk * k;
        const double k2 = kx * kx + ky * ky + kz * kz;
        s += 4.0 * M_PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2 * (1.0 - cos(kx * dx + ky * dy + kz * dz));
    }
    if (lane == 0) s -= 2.0 * alpha / sqrt(M_PI);
    return s;
}

}  // namespace fmmkmc
