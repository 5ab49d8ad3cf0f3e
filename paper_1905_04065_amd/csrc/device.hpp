// Device helpers shared by the kernels: cell indexing, neighbour wrapping,
// compile-time dispatch over the expansion order, and per-point harmonics.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "context.hpp"
#include "solid.hpp"

namespace fmmkmc {

// Global-memory view of a device pointer.  The batched kernels take their
// pointers from a replica table, where the compiler cannot see that they
// address global memory and would emit flat loads and stores (which also
// count against the LDS wait counter).  Accesses through this view are global
// ones; it must only be applied to device (global) allocations.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T *p)
{
    return (gptr<T>)p;
}

__host__ __device__ inline int64_t cell_id(int nc, int cx, int cy, int cz)
{
    return ((int64_t)cx * nc + cy) * nc + cz;
}

__host__ __device__ inline int posmod(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

__host__ __device__ inline int floordiv(int v, int n) { return v >= 0 ? v / n : -((-v + n - 1) / n); }

// fine-cell coordinate of a position component: floor(x / w), clamped to [0, nc)
__host__ __device__ inline int fine_coord(double v, double w, int nc)
{
    int c = (int)floor(v / w);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// wrap a periodic coordinate into [0, a)
__host__ __device__ inline double wrap_coord(double v, double a)
{
    double t = v - a * floor(v / a);
    return t >= a ? t - a : t;
}

// lattice site of the 2x2x2 fast path in cell-major order
__host__ __device__ inline int64_t s2_site(int nc, int i, int j, int k)
{
    return cell_id(nc, i >> 1, j >> 1, k >> 1) * 8 + ((i & 1) * 4 + (j & 1) * 2 + (k & 1));
}

// Reciprocals used by the regular recurrences at a runtime order, so that the
// recurrences carry no divisions: 1/(2k) and 1/((n+m)(n-m)) for n > m.
struct RecTables {
    double half_inv[kMaxOrder + 1];
    double rinv[kMaxOrder + 1][kMaxOrder + 1];
    constexpr RecTables() : half_inv{}, rinv{}
    {
        for (int k = 1; k <= kMaxOrder; ++k) half_inv[k] = 0.5 / k;
        for (int n = 1; n <= kMaxOrder; ++n)
            for (int m = 0; m < n; ++m) rinv[n][m] = 1.0 / (double)((n + m) * (n - m));
    }
};

// L2P (the same sum as l2p() in solid.hpp), fully unrolled, with coefficient
// k read as L(k): every load can be issued up front.
template <int P, typename T, bool SKIP0 = false, class LF>
__device__ inline T l2p_fn(LF L, T x, T y, T z)
{
    const T r2 = x * x + y * y + z * z;
    T acc0 = SKIP0 ? T(0) : L(0);
    T cm2 = T(1), cm1 = z;
    if (P >= 1) acc0 += L(slot0(1)) * z;
#pragma unroll
    for (int n = 2; n <= P; ++n) {
        const T c = ((T)(2 * n - 1) * z * cm1 - r2 * cm2) * (T)rinv(n, 0);
        acc0 += L(slot0(n)) * c;
        cm2 = cm1;
        cm1 = c;
    }
    T acc1 = T(0);
    T dr = T(1), di = T(0);
#pragma unroll
    for (int m = 1; m <= P; ++m) {
        const T f = (T)(-0.5 / m);
        const T ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        T ar = dr, ai = di;
        acc1 += L(slot_re(m, m)) * ar + L(slot_im(m, m)) * ai;
        if (m + 1 <= P) {
            T br = z * ar, bi = z * ai;
            acc1 += L(slot_re(m + 1, m)) * br + L(slot_im(m + 1, m)) * bi;
#pragma unroll
            for (int n = m + 2; n <= P; ++n) {
                const T w = (T)rinv(n, m);
                const T cr = ((T)(2 * n - 1) * z * br - r2 * ar) * w, ci = ((T)(2 * n - 1) * z * bi - r2 * ai) * w;
                acc1 += L(slot_re(n, m)) * cr + L(slot_im(n, m)) * ci;
                ar = br;
                ai = bi;
                br = cr;
                bi = ci;
            }
        }
    }
    return acc0 + T(2) * acc1;
}

// l2p_fn at G points that share one expansion and their y and z offsets (the
// same site of G consecutive x-planes of a cell): each coefficient is read
// once and used G times.
template <int P, typename T, int G, bool SKIP0 = false, class LF>
__device__ inline void l2p_fn_x(LF L, const T (&x)[G], T y, T z, T (&out)[G])
{
    T r2[G], acc0[G], acc1[G], cm2[G], cm1[G], dr[G], di[G];
    const T l0 = SKIP0 ? T(0) : L(0);
#pragma unroll
    for (int q = 0; q < G; ++q) {
        r2[q] = x[q] * x[q] + y * y + z * z;
        acc0[q] = l0;
        acc1[q] = T(0);
        cm2[q] = T(1);
        cm1[q] = z;
        dr[q] = T(1);
        di[q] = T(0);
    }
    if (P >= 1) {
        const T l = L(slot0(1));
#pragma unroll
        for (int q = 0; q < G; ++q) acc0[q] += l * z;
    }
#pragma unroll
    for (int n = 2; n <= P; ++n) {
        const T l = L(slot0(n));
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const T c = ((T)(2 * n - 1) * z * cm1[q] - r2[q] * cm2[q]) * (T)rinv(n, 0);
            acc0[q] += l * c;
            cm2[q] = cm1[q];
            cm1[q] = c;
        }
    }
#pragma unroll
    for (int m = 1; m <= P; ++m) {
        const T f = (T)(-0.5 / m);
        T ar[G], ai[G], br[G], bi[G];
        {
            const T lr = L(slot_re(m, m)), li = L(slot_im(m, m));
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const T ndr = f * (x[q] * dr[q] - y * di[q]), ndi = f * (x[q] * di[q] + y * dr[q]);
                dr[q] = ndr;
                di[q] = ndi;
                ar[q] = dr[q];
                ai[q] = di[q];
                acc1[q] += lr * ar[q] + li * ai[q];
            }
        }
        if (m + 1 <= P) {
            const T lr = L(slot_re(m + 1, m)), li = L(slot_im(m + 1, m));
#pragma unroll
            for (int q = 0; q < G; ++q) {
                br[q] = z * ar[q];
                bi[q] = z * ai[q];
                acc1[q] += lr * br[q] + li * bi[q];
            }
#pragma unroll
            for (int n = m + 2; n <= P; ++n) {
                const T w = (T)rinv(n, m);
                const T lr2 = L(slot_re(n, m)), li2 = L(slot_im(n, m));
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const T cr = ((T)(2 * n - 1) * z * br[q] - r2[q] * ar[q]) * w;
                    const T ci = ((T)(2 * n - 1) * z * bi[q] - r2[q] * ai[q]) * w;
                    acc1[q] += lr2 * cr + li2 * ci;
                    ar[q] = br[q];
                    ai[q] = bi[q];
                    br[q] = cr;
                    bi[q] = ci;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) out[q] = acc0[q] + T(2) * acc1[q];
}

// l2p_fn for the lane's fine cell of coefficient-major expansions (coefficient
// k of cell c at base[k * M + c]): each load a uniform column start plus the
// lane's 32-bit cell offset.
template <int P, typename T, bool SKIP0 = false>
__device__ inline T l2p_cell(gptr<const T> base, int64_t M, uint32_t cell, T x, T y, T z)
{
    return l2p_fn<P, T, SKIP0>([&](int k) { return (base + (int64_t)k * M)[cell]; }, x, y, z);
}

// L2P (the same sum as l2p() in solid.hpp) with the orders m >= 1 in a rolled
// loop: one column's coefficients are live at a time, so the compiler cannot
// hoist all (p+1)^2 loads at once and the caller keeps a small register
// footprint; the recurrence reciprocals come from RecTables (uniform indices).
template <int P, typename T, bool SKIP0 = false, typename PT = const T *>
__device__ inline T l2p_cols(PT L, long stride, T x, T y, T z)
{
    constexpr RecTables RT{};
    const T r2 = x * x + y * y + z * z;
    T acc0 = SKIP0 ? T(0) : L[0];
    T cm2 = T(1), cm1 = z;
    if (P >= 1) acc0 += L[slot0(1) * stride] * z;
#pragma unroll
    for (int n = 2; n <= P; ++n) {
        const T c = ((T)(2 * n - 1) * z * cm1 - r2 * cm2) * (T)RT.rinv[n][0];
        acc0 += L[slot0(n) * stride] * c;
        cm2 = cm1;
        cm1 = c;
    }
    T acc1 = T(0);
    T dr = T(1), di = T(0);
#pragma unroll 1
    for (int m = 1; m <= P; ++m) {
        const T f = -(T)RT.half_inv[m];
        const T ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        T ar = dr, ai = di;
        acc1 += L[(long)slot_re(m, m) * stride] * ar + L[(long)slot_im(m, m) * stride] * ai;
        if (m + 1 > P) break;
        T br = z * ar, bi = z * ai;
        acc1 += L[(long)slot_re(m + 1, m) * stride] * br + L[(long)slot_im(m + 1, m) * stride] * bi;
#pragma unroll 2
        for (int n = m + 2; n <= P; ++n) {
            const T w = (T)RT.rinv[n][m];
            const T zn = (T)(2 * n - 1) * z;
            const T cr = (zn * br - r2 * ar) * w, ci = (zn * bi - r2 * ai) * w;
            acc1 += L[(long)slot_re(n, m) * stride] * cr + L[(long)slot_im(n, m) * stride] * ci;
            ar = br;
            ai = bi;
            br = cr;
            bi = ci;
        }
    }
    return acc0 + T(2) * acc1;
}

// Column m (degrees n = m..p) of the regular harmonics at offset d, as L2P
// weights Wt (Psi(d) = sum_k L_k Wt[k]) and, if Km is not null, as the
// real-stored multipole of a unit charge at d (Km[k] = conj(R_k(d))).  Lanes
// m = 0..p of a group together produce the full arrays: each runs the diagonal
// recurrence to R_m^m itself (m steps) and then its column, so the dependent
// chain is at most p steps long instead of the (p+1)^2 of a single lane.
__device__ inline void harmonics_column(int p, int m, double x, double y, double z, double *Km, double *Wt)
{
    // the recurrence factors are computed, not looked up: a table indexed by the
    // lane's column is a dependent global load per step
    const double r2 = x * x + y * y + z * z;
    double ar = 1.0, ai = 0.0;
    for (int k = 1; k <= m; ++k) {
        const double f = -0.5 / (double)k;
        const double nr = f * (x * ar - y * ai), ni = f * (x * ai + y * ar);
        ar = nr;
        ai = ni;
    }
    double br = 0.0, bi = 0.0;
    for (int n = m; n <= p; ++n) {
        double cr, ci;
        if (n == m) {
            cr = ar;
            ci = ai;
        } else if (n == m + 1) {
            cr = z * ar;
            ci = z * ai;
            br = cr;
            bi = ci;
        } else {
            const double w = 1.0 / (double)((n + m) * (n - m));
            cr = ((2 * n - 1) * z * br - r2 * ar) * w;
            ci = ((2 * n - 1) * z * bi - r2 * ai) * w;
            ar = br;
            ai = bi;
            br = cr;
            bi = ci;
        }
        if (m == 0) {
            Wt[slot0(n)] = cr;
            if (Km) Km[slot0(n)] = cr;
        } else {
            Wt[slot_re(n, m)] = 2.0 * cr;
            Wt[slot_im(n, m)] = 2.0 * ci;
            if (Km) {
                Km[slot_re(n, m)] = cr;
                Km[slot_im(n, m)] = -ci;
            }
        }
    }
}

// Real-stored multipole of a unit charge at offset d (Km[k] = conj(R_k(d))) and
// the L2P weights at d (Wt[k], Psi(d) = sum L_k Wt[k]), written with stride s.
__device__ inline void unit_multipole_and_weights(int p, double x, double y, double z, double *Km, double *Wt,
                                                  int s = 1)
{
    const double r2 = x * x + y * y + z * z;
    double cm2 = 1.0, cm1 = z;
    Km[0] = 1.0;
    Wt[0] = 1.0;
    if (p >= 1) {
        Km[slot0(1) * s] = z;
        Wt[slot0(1) * s] = z;
    }
    for (int n = 2; n <= p; ++n) {
        double c = ((2 * n - 1) * z * cm1 - r2 * cm2) * rinv(n, 0);
        Km[slot0(n) * s] = c;
        Wt[slot0(n) * s] = c;
        cm2 = cm1;
        cm1 = c;
    }
    double dr = 1.0, di = 0.0;
    for (int m = 1; m <= p; ++m) {
        const double f = -0.5 / m;
        double ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        double ar = dr, ai = di, br = 0, bi = 0;
        for (int n = m; n <= p; ++n) {
            double cr, ci;
            if (n == m) {
                cr = ar;
                ci = ai;
            } else if (n == m + 1) {
                cr = z * ar;
                ci = z * ai;
                br = cr;
                bi = ci;
            } else {
                const double w = rinv(n, m);
                cr = ((2 * n - 1) * z * br - r2 * ar) * w;
                ci = ((2 * n - 1) * z * bi - r2 * ai) * w;
                ar = br;
                ai = bi;
                br = cr;
                bi = ci;
            }
            Km[slot_re(n, m) * s] = cr;
            Km[slot_im(n, m) * s] = -ci;
            Wt[slot_re(n, m) * s] = 2.0 * cr;
            Wt[slot_im(n, m) * s] = 2.0 * ci;
        }
    }
}

// Evaluate a real-stored local expansion given on the device at offset d
// (runtime order; used off the hot path).
__device__ inline double l2p_runtime(int p, const double *L, long stride, double x, double y, double z)
{
    const double r2 = x * x + y * y + z * z;
    double acc0 = L[0], acc1 = 0.0;
    double cm2 = 1.0, cm1 = z;
    if (p >= 1) acc0 += L[slot0(1) * stride] * z;
    for (int n = 2; n <= p; ++n) {
        double c = ((2 * n - 1) * z * cm1 - r2 * cm2) * rinv(n, 0);
        acc0 += L[slot0(n) * stride] * c;
        cm2 = cm1;
        cm1 = c;
    }
    double dr = 1.0, di = 0.0;
    for (int m = 1; m <= p; ++m) {
        const double f = -0.5 / m;
        double ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        double ar = dr, ai = di;
        acc1 += L[slot_re(m, m) * stride] * ar + L[slot_im(m, m) * stride] * ai;
        if (m + 1 > p) continue;
        double br = z * ar, bi = z * ai;
        acc1 += L[slot_re(m + 1, m) * stride] * br + L[slot_im(m + 1, m) * stride] * bi;
        for (int n = m + 2; n <= p; ++n) {
            const double w = rinv(n, m);
            double cr = ((2 * n - 1) * z * br - r2 * ar) * w;
            double ci = ((2 * n - 1) * z * bi - r2 * ai) * w;
            acc1 += L[slot_re(n, m) * stride] * cr + L[slot_im(n, m) * stride] * ci;
            ar = br;
            ai = bi;
            br = cr;
            bi = ci;
        }
    }
    return acc0 + 2.0 * acc1;
}

}  // namespace fmmkmc

// Expand a runtime order p (1..16) into a call of F<P>.
#define FMMKMC_DISPATCH_P(p, CALL)                                 \
    switch (p) {                                                   \
    case 1: { constexpr int P_ = 1; CALL; } break;                 \
    case 2: { constexpr int P_ = 2; CALL; } break;                 \
    case 3: { constexpr int P_ = 3; CALL; } break;                 \
    case 4: { constexpr int P_ = 4; CALL; } break;                 \
    case 5: { constexpr int P_ = 5; CALL; } break;                 \
    case 6: { constexpr int P_ = 6; CALL; } break;                 \
    case 7: { constexpr int P_ = 7; CALL; } break;                 \
    case 8: { constexpr int P_ = 8; CALL; } break;                 \
    case 9: { constexpr int P_ = 9; CALL; } break;                 \
    case 10: { constexpr int P_ = 10; CALL; } break;               \
    case 11: { constexpr int P_ = 11; CALL; } break;               \
    case 12: { constexpr int P_ = 12; CALL; } break;               \
    case 13: { constexpr int P_ = 13; CALL; } break;               \
    case 14: { constexpr int P_ = 14; CALL; } break;               \
    case 15: { constexpr int P_ = 15; CALL; } break;               \
    case 16: { constexpr int P_ = 16; CALL; } break;               \
    default: break;                                                \
    }
