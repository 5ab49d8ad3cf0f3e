// Host-side geometry tables; see tables.hpp.
#include "tables.hpp"

#include <cmath>
#include <cstring>

#include "solid.hpp"

namespace fmmkmc {

static inline int fidx(int n, int m) { return n * n + n + m; }

void regular_all(int nmax, double x, double y, double z, cplx *out)
{
    const double r2 = x * x + y * y + z * z;
    const cplx w(x, y);
    cplx diag(1.0, 0.0);
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) diag *= -w / (2.0 * m);
        out[fidx(m, m)] = diag;
        if (m + 1 <= nmax) out[fidx(m + 1, m)] = z * diag;
        for (int n = m + 2; n <= nmax; ++n)
            out[fidx(n, m)] = ((2.0 * n - 1.0) * z * out[fidx(n - 1, m)] - r2 * out[fidx(n - 2, m)]) /
                              (double)((n + m) * (n - m));
    }
    for (int n = 0; n <= nmax; ++n)
        for (int m = 1; m <= n; ++m) out[fidx(n, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(out[fidx(n, m)]);
}

void irregular_all(int nmax, double x, double y, double z, cplx *out)
{
    const double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
    const cplx w(x, y);
    cplx diag(1.0 / std::sqrt(r2), 0.0);
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) diag *= -(2.0 * m - 1.0) * w * ir2;
        out[fidx(m, m)] = diag;
        if (m + 1 <= nmax) out[fidx(m + 1, m)] = (2.0 * m + 1.0) * z * ir2 * diag;
        for (int n = m + 2; n <= nmax; ++n)
            out[fidx(n, m)] = ((2.0 * n - 1.0) * z * out[fidx(n - 1, m)] -
                               ((n - 1.0) * (n - 1.0) - (double)m * m) * out[fidx(n - 2, m)]) * ir2;
    }
    for (int n = 0; n <= nmax; ++n)
        for (int m = 1; m <= n; ++m) out[fidx(n, -m)] = ((m & 1) ? -1.0 : 1.0) * std::conj(out[fidx(n, m)]);
}

// Real matrix of a complex operator given by its coefficient g(k, l, n, m):
// out_k^l = sum_{n,m} g(k,l,n,m) in_n^m, acting on expansions with
// in_n^{-m} = (-1)^m conj(in_n^m).
template <class Coef>
static void real_matrix(int p, Coef g, double *mat)
{
    const int nt = nterms(p);
    std::memset(mat, 0, sizeof(double) * nt * nt);
    for (int k = 0; k <= p; ++k)
        for (int l = 0; l <= k; ++l)
            for (int n = 0; n <= p; ++n)
                for (int m = 0; m <= n; ++m) {
                    cplx cre, cim;  // d out_k^l / d Re(in_n^m), d / d Im(in_n^m)
                    if (m == 0) {
                        cre = g(k, l, n, 0);
                        cim = 0.0;
                    } else {
                        const double s = (m & 1) ? -1.0 : 1.0;
                        cplx a = g(k, l, n, m), b = g(k, l, n, -m);
                        cre = a + s * b;
                        cim = cplx(0.0, 1.0) * (a - s * b);
                    }
                    const int in_re = (m == 0) ? slot0(n) : slot_re(n, m);
                    if (l == 0) {
                        mat[slot0(k) * nt + in_re] = cre.real();
                        if (m > 0) mat[slot0(k) * nt + slot_im(n, m)] = cim.real();
                    } else {
                        mat[slot_re(k, l) * nt + in_re] = cre.real();
                        mat[slot_im(k, l) * nt + in_re] = cre.imag();
                        if (m > 0) {
                            mat[slot_re(k, l) * nt + slot_im(n, m)] = cim.real();
                            mat[slot_im(k, l) * nt + slot_im(n, m)] = cim.imag();
                        }
                    }
                }
}

void build_m2m(int p, double sx, double sy, double sz, double *mat)
{
    std::vector<cplx> R(nterms(p));
    regular_all(p, sx, sy, sz, R.data());
    // M_n^m(parent) = sum_{k,l} conj(R_k^l(s)) M_{n-k}^{m-l}(child)
    real_matrix(
        p,
        [&](int n, int m, int nn, int mm) -> cplx {
            int k = n - nn, l = m - mm;
            if (k < 0 || l < -k || l > k) return 0.0;
            return std::conj(R[fidx(k, l)]);
        },
        mat);
}

void build_l2l(int p, double sx, double sy, double sz, double *mat)
{
    std::vector<cplx> R(nterms(p));
    regular_all(p, sx, sy, sz, R.data());
    // L'_j^i = sum_{k >= j, l} L_k^l conj(R_{k-j}^{l-i}(s)), s = new - old centre
    real_matrix(
        p,
        [&](int j, int i, int k, int l) -> cplx {
            int dk = k - j, dl = l - i;
            if (dk < 0 || dl < -dk || dl > dk) return 0.0;
            return std::conj(R[fidx(dk, dl)]);
        },
        mat);
}

void build_m2l(int p, double dx, double dy, double dz, double *mat)
{
    std::vector<cplx> I(nterms(2 * p));
    irregular_all(2 * p, dx, dy, dz, I.data());
    // L_k^l = (-1)^k sum_{n,m} M_n^m I_{n+k}^{m+l}(d), d = target - source
    real_matrix(
        p,
        [&](int k, int l, int n, int m) -> cplx { return ((k & 1) ? -1.0 : 1.0) * I[fidx(n + k, m + l)]; },
        mat);
}

// regularised upper incomplete gamma Q(s + 1/2, x) for s = 0..smax
static void gamma_half(int smax, double x, double *Q)
{
    // Gamma(1/2, x) = sqrt(pi) erfc(sqrt x); Gamma(a+1, x) = a Gamma(a, x) + x^a e^-x
    double G = std::sqrt(M_PI) * std::erfc(std::sqrt(x)), Gfull = std::sqrt(M_PI);
    double a = 0.5;
    for (int s = 0; s <= smax; ++s) {
        Q[s] = G / Gfull;
        G = a * G + std::pow(x, a) * std::exp(-x);
        Gfull *= a;
        a += 1.0;
    }
}

void lattice_sums(int smax, double a, cplx *S)
{
    const int nt = nterms(smax);
    std::vector<cplx> acc(nt, 0.0), Rv(nt);
    std::vector<double> Q(smax + 1);
    std::vector<double> fac(2 * smax + 2, 1.0);
    for (int i = 1; i < (int)fac.size(); ++i) fac[i] = fac[i - 1] * i;
    const double alpha = std::sqrt(M_PI);
    const int nmax = 6;
    std::vector<double> gfull(smax + 1);
    {
        double g = std::sqrt(M_PI), aa = 0.5;
        for (int s = 0; s <= smax; ++s) {
            gfull[s] = g;
            g *= aa;
            aa += 1.0;
        }
    }
    // sum over Z^3 \ 0 of I_s^t(nu) = Y(nu) / |nu|^(2s+1) with Y = (s-|t|)!(s+|t|)! R_s^t
    for (int i = -nmax; i <= nmax; ++i)
        for (int j = -nmax; j <= nmax; ++j)
            for (int k = -nmax; k <= nmax; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                const double rr = (double)(i * i + j * j + k * k);
                regular_all(smax, i, j, k, Rv.data());
                gamma_half(smax, alpha * alpha * rr, Q.data());
                const double ek = std::exp(-M_PI * M_PI * rr / (alpha * alpha)) / rr;
                for (int s = 3; s <= smax; s += 1) {
                    if (s & 1) continue;
                    const double real_w = Q[s] / std::pow(rr, s + 0.5);
                    const double recip_w = ((s / 2) & 1 ? -1.0 : 1.0) * std::pow(M_PI, s - 0.5) / gfull[s] * ek;
                    for (int t = -s; t <= s; ++t) {
                        const int at = t < 0 ? -t : t;
                        const cplx Y = fac[s - at] * fac[s + at] * Rv[fidx(s, t)];
                        acc[fidx(s, t)] += Y * (real_w + recip_w);
                    }
                }
            }
    // minus the 26 copies of V_box
    std::vector<cplx> Iv(nt);
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                irregular_all(smax, i, j, k, Iv.data());
                for (int s = 3; s <= smax; ++s) {
                    if (s & 1) continue;
                    for (int t = -s; t <= s; ++t) acc[fidx(s, t)] -= Iv[fidx(s, t)];
                }
            }
    for (int s = 0; s <= smax; ++s)
        for (int t = -s; t <= s; ++t)
            S[fidx(s, t)] = (s < 3 || (s & 1)) ? cplx(0.0) : acc[fidx(s, t)] * std::pow(a, -(s + 1.0));
}

void build_far_operator(int p, double a, double *mat)
{
    std::vector<cplx> S(nterms(2 * p));
    lattice_sums(2 * p, a, S.data());
    // copies at c + a nu seen from c: d = -a nu; the sum is even in nu for even s
    real_matrix(
        p,
        [&](int k, int l, int n, int m) -> cplx { return ((k & 1) ? -1.0 : 1.0) * S[fidx(n + k, m + l)]; },
        mat);
    if (p >= 1) {
        const int nt = nterms(p);
        const double c = 4.0 * M_PI / (3.0 * a * a * a);
        mat[slot0(1) * nt + slot0(1)] += -c;
        mat[slot_re(1, 1) * nt + slot_re(1, 1)] += -2.0 * c;
        mat[slot_im(1, 1) * nt + slot_im(1, 1)] += 2.0 * c;
    }
}

double build_cheb_map(int p, double a, double *G)
{
    const int nt = nterms(p), q = p + 1;
    const double rho = 0.5 * a;
    std::vector<double> xi(q), w(nt);
    for (int j = 0; j < q; ++j) xi[j] = (p == 0) ? 0.0 : std::cos(M_PI * j / p);
    // samples f[j1][j2][j3][k]
    std::vector<double> f((size_t)q * q * q * nt), g((size_t)q * q * q * nt);
    for (int j1 = 0; j1 < q; ++j1)
        for (int j2 = 0; j2 < q; ++j2)
            for (int j3 = 0; j3 < q; ++j3) {
                l2p_weights(p, rho * xi[j1], rho * xi[j2], rho * xi[j3], w.data());
                std::memcpy(&f[(((size_t)j1 * q + j2) * q + j3) * nt], w.data(), sizeof(double) * nt);
            }
    // DCT-I along each axis: c_a = (2/p) sum_j'' f_j cos(pi a j / p), halved for a = 0, p
    auto dct_axis = [&](int axis, const std::vector<double> &in, std::vector<double> &out) {
        std::fill(out.begin(), out.end(), 0.0);
        for (int i1 = 0; i1 < q; ++i1)
            for (int i2 = 0; i2 < q; ++i2)
                for (int aa = 0; aa < q; ++aa) {
                    for (int j = 0; j < q; ++j) {
                        double wj = (p == 0) ? 1.0 : 2.0 / p * ((j == 0 || j == p) ? 0.5 : 1.0) *
                                                          std::cos(M_PI * aa * j / (double)p);
                        if (p > 0 && (aa == 0 || aa == p)) wj *= 0.5;
                        int src[3], dst[3];
                        src[axis] = j;
                        dst[axis] = aa;
                        int o1 = (axis == 0) ? 1 : 0, o2 = (axis == 2) ? 1 : 2;
                        src[o1] = dst[o1] = i1;
                        src[o2] = dst[o2] = i2;
                        const double *fi = &in[(((size_t)src[0] * q + src[1]) * q + src[2]) * nt];
                        double *go = &out[(((size_t)dst[0] * q + dst[1]) * q + dst[2]) * nt];
                        for (int k = 0; k < nt; ++k) go[k] += wj * fi[k];
                    }
                }
    };
    dct_axis(0, f, g);
    dct_axis(1, g, f);
    dct_axis(2, f, g);
    double leak = 0.0;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j)
            for (int k = 0; k < q; ++k) {
                double *src = &g[(((size_t)i * q + j) * q + k) * nt];
                double *dst = &G[(((size_t)i * q + j) * q + k) * nt];
                if (i + j + k > p) {
                    for (int t = 0; t < nt; ++t) {
                        leak = std::fmax(leak, std::fabs(src[t]));
                        dst[t] = 0.0;
                    }
                } else {
                    std::memcpy(dst, src, sizeof(double) * nt);
                }
            }
    return leak;
}

void build_s2_tables(int p, double h, double *Y2, double *T2)
{
    const int nt = nterms(p);
    for (int u = 0; u < 8; ++u) {
        const int lx = u >> 2, ly = (u >> 1) & 1, lz = u & 1;
        l2p_weights(p, (lx - 0.5) * h, (ly - 0.5) * h, (lz - 0.5) * h, Y2 + u * nt);
        for (int nb = 0; nb < 27; ++nb) {
            const int dx = nb / 9 - 1, dy = (nb / 3) % 3 - 1, dz = nb % 3 - 1;
            for (int v = 0; v < 8; ++v) {
                const int mx = v >> 2, my = (v >> 1) & 1, mz = v & 1;
                const double ex = 2 * dx + mx - lx, ey = 2 * dy + my - ly, ez = 2 * dz + mz - lz;
                const double r = h * std::sqrt(ex * ex + ey * ey + ez * ez);
                T2[u * 216 + nb * 8 + v] = (r == 0.0) ? 0.0 : 1.0 / r;
            }
        }
    }
}

}  // namespace fmmkmc
