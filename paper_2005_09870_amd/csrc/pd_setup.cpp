// pd_setup.cpp -- host-side set-up of a solve: the Symmlet filter bank, the
// Operator-1 tap table and its product-convolution expansion (Escande & Weiss,
// arXiv:2005.09870, Sections 2.1, 3.3.3, 4.1, 4.2).  Plain C++, no GPU code.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "pd.h"

namespace {

using cld = std::complex<long double>;

// Roots of the real polynomial c[0] + c[1] x + ... + c[n] x^n by the
// Weierstrass (Durand-Kerner) simultaneous iteration, then Newton polishing.
std::vector<cld> poly_roots(const std::vector<long double> &c)
{
    const int n = (int)c.size() - 1;
    std::vector<cld> a(n + 1);
    for (int i = 0; i <= n; ++i) a[i] = c[i] / c[n];  // monic
    auto eval = [&](cld x) {
        cld v = 1.0L;
        for (int i = n - 1; i >= 0; --i) v = v * x + a[i];
        return v;
    };
    std::vector<cld> r(n);
    const cld seed(0.4L, 0.9L);
    for (int i = 0; i < n; ++i) r[i] = std::pow(seed, i);
    for (int it = 0; it < 2000; ++it) {
        long double delta = 0.0L;
        for (int i = 0; i < n; ++i) {
            cld den = 1.0L;
            for (int j = 0; j < n; ++j)
                if (j != i) den *= (r[i] - r[j]);
            cld step = eval(r[i]) / den;
            r[i] -= step;
            delta = std::max(delta, std::abs(step));
        }
        if (delta < 1e-30L) break;
    }
    for (int i = 0; i < n; ++i) {  // Newton polish on the monic polynomial
        for (int it = 0; it < 5; ++it) {
            cld p = 1.0L, dp = 0.0L;
            for (int k = n - 1; k >= 0; --k) {
                dp = dp * r[i] + p;
                p = p * r[i] + a[k];
            }
            if (std::abs(dp) == 0.0L) break;
            r[i] -= p / dp;
        }
    }
    return r;
}

std::vector<cld> poly_from_roots(const std::vector<cld> &roots)
{
    std::vector<cld> p(1, cld(1.0L));  // increasing powers
    for (const cld &z : roots) {
        std::vector<cld> q(p.size() + 1, cld(0.0L));
        for (size_t i = 0; i < p.size(); ++i) {
            q[i + 1] += p[i];
            q[i] -= z * p[i];
        }
        p.swap(q);
    }
    return p;
}

// Squared deviation of the unwrapped phase of q(e^{-iw}) from its least-squares
// straight line over w in [0, pi] (4097 samples).
long double phase_nonlinearity(const std::vector<cld> &q)
{
    const int S = 4097;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> w(S), ph(S);
    long double prev = 0.0L, offset = 0.0L;
    for (int s = 0; s < S; ++s) {
        w[s] = pi * s / (S - 1);
        cld e = std::polar(1.0L, -w[s]);
        cld v = 0.0L, ek = 1.0L;
        for (const cld &c : q) {
            v += c * ek;
            ek *= e;
        }
        long double a = std::arg(v);
        if (s > 0) {
            long double d = a - prev;
            if (d > pi) offset -= 2 * pi;
            if (d < -pi) offset += 2 * pi;
        }
        prev = a;
        ph[s] = a + offset;
    }
    long double sw = 0, sp = 0, sww = 0, swp = 0;
    for (int s = 0; s < S; ++s) {
        sw += w[s];
        sp += ph[s];
        sww += w[s] * w[s];
        swp += w[s] * ph[s];
    }
    long double b = (S * swp - sw * sp) / (S * sww - sw * sw);
    long double a0 = (sp - b * sw) / S;
    long double r2 = 0;
    for (int s = 0; s < S; ++s) {
        long double e = ph[s] - a0 - b * w[s];
        r2 += e * e;
    }
    return r2;
}

// Inverse error function by Newton's method on erf.
long double erfinv_ld(long double y)
{
    long double x = 0.0L;
    const long double c = 2.0L / std::sqrt(3.141592653589793238462643383279502884L);
    for (int it = 0; it < 100; ++it) {
        long double f = std::erf(x) - y;
        long double d = c * std::exp(-x * x);
        long double step = f / d;
        x -= step;
        if (std::fabs(step) < 1e-18L) break;
    }
    return x;
}

}  // namespace

extern "C" int pd_symmlet(int32_t moments, double *h_out)
{
    if (!h_out || moments < 1 || moments > 10) return PD_ERR_ARG;
    const int M = moments;
    if (M == 1) {
        h_out[0] = h_out[1] = 1.0 / std::sqrt(2.0);
        return PD_OK;
    }
    // Daubechies: |m0(w)|^2 = cos^{2M}(w/2) P(sin^2(w/2)), P(y) = sum_{k<M} C(M-1+k,k) y^k.
    std::vector<long double> P(M);
    for (int k = 0; k < M; ++k) {
        long double b = 1.0L;  // binomial C(M-1+k, k)
        for (int j = 1; j <= k; ++j) b = b * (M - 1 + j) / j;
        P[k] = b;
    }
    std::vector<cld> yr = poly_roots(P);
    // Each root y gives z + 1/z = 2 - 4y; keep the root inside the unit circle.
    // Group conjugate pairs (one group per real root or per conjugate pair).
    std::vector<std::vector<cld>> groups;
    std::vector<bool> used(yr.size(), false);
    for (size_t a = 0; a < yr.size(); ++a) {
        if (used[a]) continue;
        used[a] = true;
        cld b = 2.0L - 4.0L * yr[a];
        cld sq = std::sqrt(b * b - 4.0L);
        cld z1 = (b + sq) / 2.0L, z2 = (b - sq) / 2.0L;
        cld zin = std::abs(z1) < 1.0L ? z1 : z2;
        if (std::fabs(yr[a].imag()) > 1e-12L * std::max(1.0L, std::abs(yr[a]))) {
            size_t best = a;
            long double bd = 1e300L;
            for (size_t q = 0; q < yr.size(); ++q)
                if (!used[q] && std::abs(yr[q] - std::conj(yr[a])) < bd) {
                    bd = std::abs(yr[q] - std::conj(yr[a]));
                    best = q;
                }
            used[best] = true;
            groups.push_back({zin, std::conj(zin)});
        } else {
            groups.push_back({cld(zin.real(), 0.0L)});
        }
    }
    // Enumerate inside/outside choices (group 0 held inside: each mirror pair
    // once); keep the most nearly linear phase.
    const int G = (int)groups.size();
    long double best_score = 0.0L;
    std::vector<cld> best_roots;
    for (int mask = 0; mask < (1 << (G - 1)); ++mask) {
        std::vector<cld> roots;
        for (int g = 0; g < G; ++g) {
            bool outside = g > 0 && ((mask >> (g - 1)) & 1);
            for (const cld &z : groups[g]) roots.push_back(outside ? 1.0L / z : z);
        }
        std::vector<cld> q = poly_from_roots(roots);
        long double s = phase_nonlinearity(q);
        if (best_roots.empty() || s < best_score) {
            best_score = s;
            best_roots = roots;
        }
    }
    std::vector<cld> q = poly_from_roots(best_roots);
    long double qs = 0.0L;
    for (const cld &c : q) qs += c.real();
    // h = sqrt(2) * ((1+z)/2)^M * q(z)/q(1)
    std::vector<long double> lo(1, 1.0L);
    for (int m = 0; m < M; ++m) {
        std::vector<long double> t(lo.size() + 1, 0.0L);
        for (size_t i = 0; i < lo.size(); ++i) {
            t[i] += 0.5L * lo[i];
            t[i + 1] += 0.5L * lo[i];
        }
        lo.swap(t);
    }
    std::vector<long double> h(lo.size() + q.size() - 1, 0.0L);
    for (size_t i = 0; i < lo.size(); ++i)
        for (size_t j = 0; j < q.size(); ++j) h[i + j] += lo[i] * q[j].real() / qs;
    const long double r2 = std::sqrt(2.0L);
    long double cen = 0.0L;
    for (size_t n = 0; n < h.size(); ++n) {
        h[n] *= r2;
        cen += n * h[n] * h[n];
    }
    // mirror image: energy centroid in the upper half of [0, 2M-1]
    if (cen < (h.size() - 1) / 2.0L) std::reverse(h.begin(), h.end());
    for (int n = 0; n < 2 * M; ++n) h_out[n] = (double)h[n];
    return PD_OK;
}

extern "C" int pd_op1_taps(int32_t n2, double sigma_max, double mass, int32_t *radius,
                           double *taps_out)
{
    if (!radius || n2 < 1 || !(sigma_max >= 0.0) || !(mass > 0.0 && mass < 1.0))
        return PD_ERR_ARG;
    // square window keeping `mass` of a 2-D isotropic Gaussian: per-axis mass
    // sqrt(mass), half-width sigma * sqrt(2) * erfinv(sqrt(mass)).
    const long double k = std::sqrt(2.0L) * erfinv_ld(std::sqrt((long double)mass));
    std::vector<int> rr(n2);
    std::vector<long double> sig(n2);
    int R = 0;
    for (int i = 0; i < n2; ++i) {
        sig[i] = n2 > 1 ? (long double)sigma_max * i / (n2 - 1) : 0.0L;
        rr[i] = sig[i] > 0.0L ? (int)std::ceil(sig[i] * k) : 0;
        R = std::max(R, rr[i]);
    }
    *radius = R;
    if (!taps_out) return PD_OK;
    const int W = 2 * R + 1;
    for (int i = 0; i < n2; ++i) {
        double *row = taps_out + (size_t)i * W;
        for (int d = 0; d < W; ++d) row[d] = 0.0;
        if (rr[i] == 0) {
            row[R] = 1.0;
            continue;
        }
        long double s = 0.0L;
        std::vector<long double> p(2 * rr[i] + 1);
        for (int d = -rr[i]; d <= rr[i]; ++d) {
            p[d + rr[i]] = std::exp(-(long double)d * d / (2.0L * sig[i] * sig[i]));
            s += p[d + rr[i]];
        }
        for (int d = -rr[i]; d <= rr[i]; ++d) row[R + d] = (double)(p[d + rr[i]] / s);
    }
    return PD_OK;
}

// ---------------------------------------------------------------------------
// Product-convolution expansion of Operator 1 by a randomized SVD of its SVIR
// (Section 3.3.3; the range finder with subspace iteration and the direct SVD
// of the projected matrix of Halko, Martinsson and Tropp).  S has one row per
// offset (d2, d1) of the (2R+1)^2 window, row-major, and one column per source
// row y (Operator 1's response depends on the source row only): S[(a, b), y] =
// p_y[a] p_y[b], p_y the row's profile.  Only products with S and S^T are used.
// ---------------------------------------------------------------------------
namespace {

// SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator.
uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// Standard normal number i of stream `seed` (Box-Muller on two uniforms in (0, 1)).
double gauss(uint64_t seed, uint64_t i)
{
    const uint64_t a = splitmix64(seed ^ splitmix64(2 * i)), b = splitmix64(seed ^ splitmix64(2 * i + 1));
    const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53, u2 = ((double)(b >> 11) + 0.5) * 0x1.0p-53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925286766559 * u2);
}

struct Svir {
    const double *taps;
    int n2, W;
    int rows() const { return W * W; }
    // out[W W] = S x, x[n2]
    void apply(const double *x, double *out) const
    {
        std::fill(out, out + rows(), 0.0);
        for (int y = 0; y < n2; ++y) {
            if (x[y] == 0.0) continue;
            const double *p = taps + (size_t)y * W;
            for (int a = 0; a < W; ++a) {
                const double t = x[y] * p[a];
                for (int b = 0; b < W; ++b) out[a * W + b] += t * p[b];
            }
        }
    }
    // out[n2] = S^T q, q[W W]
    void apply_t(const double *q, double *out) const
    {
        for (int y = 0; y < n2; ++y) {
            const double *p = taps + (size_t)y * W;
            double s = 0.0;
            for (int a = 0; a < W; ++a) {
                double r = 0.0;
                for (int b = 0; b < W; ++b) r += q[a * W + b] * p[b];
                s += p[a] * r;
            }
            out[y] = s;
        }
    }
};

double dot(const double *a, const double *b, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

// Orthonormal basis of the k columns of Y (column j at Y + j n) by modified
// Gram-Schmidt, each column orthogonalised twice; a column left with at most
// 1e-13 of its norm (Y rank-deficient) becomes zero.  Returns the rank.
int orthonormalise(std::vector<double> &Y, int n, int k)
{
    int rank = 0;
    for (int j = 0; j < k; ++j) {
        double *c = Y.data() + (size_t)j * n;
        const double n0 = std::sqrt(dot(c, c, n));
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                const double *q = Y.data() + (size_t)i * n;
                const double r = dot(q, c, n);
                for (int t = 0; t < n; ++t) c[t] -= r * q[t];
            }
        const double nr = std::sqrt(dot(c, c, n));
        if (n0 == 0.0 || nr <= 1e-13 * n0) {
            std::fill(c, c + n, 0.0);
            continue;
        }
        for (int t = 0; t < n; ++t) c[t] /= nr;
        ++rank;
    }
    return rank;
}

// One-sided Jacobi (Hestenes): rotates the k columns of G (column j at G + j n)
// until they are mutually orthogonal, accumulating the rotations in J (k x k,
// column-major, starts as the identity).  Afterwards G = G0 J has orthogonal
// columns whose norms are the singular values of G0.
void jacobi_svd(std::vector<double> &G, int n, int k, std::vector<double> &J)
{
    J.assign((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) J[(size_t)j * k + j] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = i + 1; j < k; ++j) {
                double *gi = G.data() + (size_t)i * n, *gj = G.data() + (size_t)j * n;
                const double a = dot(gi, gi, n), b = dot(gj, gj, n), c = dot(gi, gj, n);
                if (c == 0.0 || std::fabs(c) <= 1e-15 * std::sqrt(a * b)) continue;
                off = std::max(off, std::fabs(c) / std::sqrt(a * b));
                // the rotation that zeroes the (i, j) entry of the 2 x 2 Gram matrix
                const double zeta = (b - a) / (2.0 * c);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int r = 0; r < n; ++r) {
                    const double x = gi[r], y = gj[r];
                    gi[r] = cs * x - sn * y;
                    gj[r] = sn * x + cs * y;
                }
                double *ji = J.data() + (size_t)i * k, *jj = J.data() + (size_t)j * k;
                for (int r = 0; r < k; ++r) {
                    const double x = ji[r], y = jj[r];
                    ji[r] = cs * x - sn * y;
                    jj[r] = sn * x + cs * y;
                }
            }
        if (off <= 1e-15) break;
    }
}

}  // namespace

extern "C" int pd_pc_expansion(const double *taps, int32_t n2, int32_t radius, int32_t terms, int32_t oversample,
                               int32_t power_iters, uint64_t seed, double *u_out, double *v_out, double *sv_out,
                               int32_t *terms_out)
{
    if (!taps || !u_out || !v_out || !terms_out || n2 < 1 || radius < 0 || radius > 64 || terms < 1 ||
        oversample < 0 || oversample > 64 || power_iters < 0 || power_iters > 16)
        return PD_ERR_ARG;
    const int W = 2 * radius + 1, M = W * W;
    const Svir S{taps, n2, W};
    const int k = std::min({terms + oversample, n2, M});
    // range finder: Y = S Omega, Omega n2 x k Gaussian; then power_iters rounds
    // of Q <- orth(S orth(S^T Q))
    std::vector<double> Y((size_t)M * k), Z((size_t)n2 * k), om(n2);
    for (int j = 0; j < k; ++j) {
        for (int y = 0; y < n2; ++y) om[y] = gauss(seed, (uint64_t)j * n2 + y);
        S.apply(om.data(), Y.data() + (size_t)j * M);
    }
    int rank = orthonormalise(Y, M, k);
    for (int it = 0; it < power_iters && rank > 0; ++it) {
        for (int j = 0; j < k; ++j) S.apply_t(Y.data() + (size_t)j * M, Z.data() + (size_t)j * n2);
        orthonormalise(Z, n2, k);
        for (int j = 0; j < k; ++j) S.apply(Z.data() + (size_t)j * n2, Y.data() + (size_t)j * M);
        rank = orthonormalise(Y, M, k);
    }
    // B = Q^T S (k x n2), held as its transpose G = S^T Q (column j = S^T q_j);
    // B = J Sigma V^T from the one-sided Jacobi of G, so u = Q J
    std::vector<double> G((size_t)n2 * k), J;
    for (int j = 0; j < k; ++j) S.apply_t(Y.data() + (size_t)j * M, G.data() + (size_t)j * n2);
    jacobi_svd(G, n2, k, J);
    std::vector<double> sv(k);
    std::vector<int> ord(k);
    for (int j = 0; j < k; ++j) {
        sv[j] = std::sqrt(dot(G.data() + (size_t)j * n2, G.data() + (size_t)j * n2, n2));
        ord[j] = j;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sv[a] > sv[b]; });
    int m = 0;
    while (m < std::min(terms, k) && sv[ord[m]] > 0.0 && sv[ord[m]] > 1e-14 * sv[ord[0]]) ++m;
    std::vector<double> u(M);
    for (int t = 0; t < m; ++t) {
        const int j = ord[t];
        std::fill(u.begin(), u.end(), 0.0);
        for (int i = 0; i < k; ++i) {
            const double c = J[(size_t)j * k + i];
            const double *q = Y.data() + (size_t)i * M;
            for (int r = 0; r < M; ++r) u[r] += c * q[r];
        }
        const double nu = std::sqrt(dot(u.data(), u.data(), M));
        int big = 0;  // sign: the entry of largest magnitude is positive
        for (int r = 1; r < M; ++r)
            if (std::fabs(u[r]) > std::fabs(u[big])) big = r;
        const double sc = (u[big] < 0.0 ? -1.0 : 1.0) / nu;
        for (int r = 0; r < M; ++r) u_out[(size_t)t * M + r] = u[r] * sc;
        S.apply_t(u_out + (size_t)t * M, v_out + (size_t)t * n2);  // v_t(y) = <S(., y), u_t>
        if (sv_out) sv_out[t] = sv[j];
    }
    *terms_out = m;
    return m > 0 ? PD_OK : PD_ERR_ARG;
}

extern "C" const char *pd_strerror(int32_t status)
{
    switch (status) {
    case PD_OK: return "ok";
    case PD_ERR_ARG: return "invalid argument (null pointer, bad enum or count)";
    case PD_ERR_SHAPE: return "invalid shape (sizes must be divisible by 2^levels)";
    case PD_ERR_WORKSPACE: return "workspace too small";
    case PD_ERR_TAU: return "step size must be finite and > 0";
    case PD_ERR_NONFINITE: return "non-finite value in the iteration";
    case PD_ERR_HIP: return "HIP runtime error";
    case PD_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}
