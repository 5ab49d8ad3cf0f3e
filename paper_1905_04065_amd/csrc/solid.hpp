// Regular and irregular solid harmonics for the FMM operators (host and device).
//
// Convention (complex, all |m| <= n):
//   R_0^0 = 1,   R_m^m = -(x + i y)/(2m) R_{m-1}^{m-1},
//   (n+m)(n-m) R_n^m = (2n-1) z R_{n-1}^m - r^2 R_{n-2}^m,
//   I_0^0 = 1/r, I_m^m = -(2m-1)(x + i y)/r^2 I_{m-1}^{m-1},
//   r^2 I_n^m = (2n-1) z I_{n-1}^m - ((n-1)^2 - m^2) I_{n-2}^m,
//   R_n^{-m} = (-1)^m conj(R_n^m), I_n^{-m} = (-1)^m conj(I_n^m).
// With these, 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x|,
// R_n^m(x + y) = sum_{k,l} R_k^l(x) R_{n-k}^{m-l}(y), and
// I_n^m(x - y) = sum_{k,l} conj(R_k^l(y)) I_{n+k}^{m+l}(x).
//
// Expansions about a centre c (the Phi and Psi of Eq. (multipole_local_expansion)
// in this basis):
//   multipole  M_n^m = sum_i q_i conj(R_n^m(y_i - c)),  Phi(x) = sum M_n^m I_n^m(x - c)
//   local      Psi(x) = sum L_n^m conj(R_n^m(x - c))
//   P2L of q at y:  L_n^m = q I_n^m(y - c)
// A real potential has L_n^{-m} = (-1)^m conj(L_n^m), so (p+1)^2 reals store an
// expansion: slot n^2 holds the (real) m = 0 coefficient and slots n^2 + 2m - 1,
// n^2 + 2m hold Re and Im of the m > 0 coefficient.  Then
//   Psi(u) = sum_n [ L_n^0 R_n^0(u) + 2 sum_{m>0} (Re L Re R + Im L Im R) ].
#pragma once

#include <hip/hip_runtime.h>

namespace fmmkmc {

__host__ __device__ constexpr int nterms(int p) { return (p + 1) * (p + 1); }
__host__ __device__ constexpr int slot0(int n) { return n * n; }
__host__ __device__ constexpr int slot_re(int n, int m) { return n * n + 2 * m - 1; }
__host__ __device__ constexpr int slot_im(int n, int m) { return n * n + 2 * m; }

// 1 / ((n+m)(n-m)) for the regular recurrence, n > m >= 0
__host__ __device__ constexpr double rinv(int n, int m) { return 1.0 / (double)((n + m) * (n - m)); }

// Evaluate a real-stored local expansion at offset u (Psi(u) above).
// L[k * stride] is coefficient k; T is float or double.  With SKIP0 the
// constant term L[0] is left out (the caller adds it in higher precision).
template <int P, typename T, bool SKIP0 = false>
__host__ __device__ inline T l2p(const T *L, long stride, T x, T y, T z)
{
    const T r2 = x * x + y * y + z * z;
    // m = 0 column
    T acc0 = SKIP0 ? T(0) : L[0];
    T cm2 = T(1), cm1 = z;
    if (P >= 1) acc0 += L[slot0(1) * stride] * z;
#pragma unroll
    for (int n = 2; n <= P; ++n) {
        T c = ((T)(2 * n - 1) * z * cm1 - r2 * cm2) * (T)rinv(n, 0);
        acc0 += L[slot0(n) * stride] * c;
        cm2 = cm1;
        cm1 = c;
    }
    T acc1 = T(0);
    T dr = T(1), di = T(0);
#pragma unroll
    for (int m = 1; m <= P; ++m) {
        const T f = (T)(-0.5 / m);
        T ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        T ar = dr, ai = di;              // R_m^m
        acc1 += L[slot_re(m, m) * stride] * ar + L[slot_im(m, m) * stride] * ai;
        if (m + 1 <= P) {
            T br = z * ar, bi = z * ai;  // R_{m+1}^m
            acc1 += L[slot_re(m + 1, m) * stride] * br + L[slot_im(m + 1, m) * stride] * bi;
#pragma unroll
            for (int n = m + 2; n <= P; ++n) {
                const T w = (T)rinv(n, m);
                T cr = ((T)(2 * n - 1) * z * br - r2 * ar) * w;
                T ci = ((T)(2 * n - 1) * z * bi - r2 * ai) * w;
                acc1 += L[slot_re(n, m) * stride] * cr + L[slot_im(n, m) * stride] * ci;
                ar = br;
                ai = bi;
                br = cr;
                bi = ci;
            }
        }
    }
    return acc0 + T(2) * acc1;
}

// Real-stored regular harmonics with the L2P weights folded in:
// out[k] such that Psi(u) = sum_k L[k] out[k].
template <typename T>
__host__ __device__ inline void l2p_weights(int p, T x, T y, T z, T *out)
{
    const T r2 = x * x + y * y + z * z;
    T cm2 = T(1), cm1 = z;
    out[0] = T(1);
    if (p >= 1) out[slot0(1)] = z;
    for (int n = 2; n <= p; ++n) {
        T c = ((T)(2 * n - 1) * z * cm1 - r2 * cm2) * (T)rinv(n, 0);
        out[slot0(n)] = c;
        cm2 = cm1;
        cm1 = c;
    }
    T dr = T(1), di = T(0);
    for (int m = 1; m <= p; ++m) {
        const T f = (T)(-0.5 / m);
        T ndr = f * (x * dr - y * di), ndi = f * (x * di + y * dr);
        dr = ndr;
        di = ndi;
        T ar = dr, ai = di;
        out[slot_re(m, m)] = T(2) * ar;
        out[slot_im(m, m)] = T(2) * ai;
        if (m + 1 > p) continue;
        T br = z * ar, bi = z * ai;
        out[slot_re(m + 1, m)] = T(2) * br;
        out[slot_im(m + 1, m)] = T(2) * bi;
        for (int n = m + 2; n <= p; ++n) {
            const T w = (T)rinv(n, m);
            T cr = ((T)(2 * n - 1) * z * br - r2 * ar) * w;
            T ci = ((T)(2 * n - 1) * z * bi - r2 * ai) * w;
            out[slot_re(n, m)] = T(2) * cr;
            out[slot_im(n, m)] = T(2) * ci;
            ar = br;
            ai = bi;
            br = cr;
            bi = ci;
        }
    }
}

// Regular harmonics column m (n = m..p) at (x, y, z): re[n-m], im[n-m] = R_n^m.
// dr, di must hold R_m^m on entry (the diagonal, built by the caller).
__host__ __device__ inline void regular_column(int p, int m, double x, double y, double z, double dr, double di,
                                               double *re, double *im)
{
    const double r2 = x * x + y * y + z * z;
    double ar = dr, ai = di;
    re[0] = ar;
    im[0] = ai;
    if (m + 1 > p) return;
    double br = z * ar, bi = z * ai;
    re[1] = br;
    im[1] = bi;
    for (int n = m + 2; n <= p; ++n) {
        const double w = rinv(n, m);
        double cr = ((2 * n - 1) * z * br - r2 * ar) * w;
        double ci = ((2 * n - 1) * z * bi - r2 * ai) * w;
        re[n - m] = cr;
        im[n - m] = ci;
        ar = br;
        ai = bi;
        br = cr;
        bi = ci;
    }
}

}  // namespace fmmkmc
