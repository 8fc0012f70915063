/*
 * oracle.c -- the oracle: a plain, slow, FP64 CPU implementation of the
 * wavelet-l1 deblurring energy of Escande & Weiss (arXiv:2005.09870) and of
 * the FISTA iteration that minimises it in its spatial-operator form.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or constant generator with the GPU library; every loop
 * below is written straight from the definition it cites.
 *
 * Conventions (all arrays row-major, x1 = fastest axis, periodic boundary):
 *   image / coefficient plane : a[i2 * n1 + i1], i1 in [0,n1), i2 in [0,n2)
 *   C channels                 : planar, channel c at offset c * n1 * n2
 *   wavelet coefficients       : Mallat layout in an n2 x n1 plane (after
 *                                level 1: LL top-left, high-in-x1 top-right,
 *                                high-in-x2 bottom-left, high-in-both
 *                                bottom-right; recursively on LL).
 *
 * Citations refer to the paper's sections and equations.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the parallel loops below use. */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int pmod(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* High-pass filter of Section 2.1: g[k] = (-1)^(1-k) h[1-k], defined for
 * k in [2-L, 1] when h is supported on [0, L-1]. */
static double gtap(const double *h, int L, int k)
{
    int m = 1 - k; /* index into h, in [0, L-1] */
    if (m < 0 || m >= L) return 0.0;
    return (m % 2 == 0 ? 1.0 : -1.0) * h[m];
}

/* ------------------------------------------------------------------------
 * One level of the periodic 1-D orthogonal wavelet transform (Section 2.1).
 * Scaling and wavelet coefficients at the coarser scale are inner products
 * with phi_{j,l} = sum_n h[n-2l] phi_{j+1,n} and psi_{j,l} = sum_n g[n-2l]
 * phi_{j+1,n}, i.e.
 *     lo[l] = sum_n h[n - 2l] in[n],   hi[l] = sum_n g[n - 2l] in[n],
 * with n taken modulo the signal length (circular boundary, Section 2).
 * ---------------------------------------------------------------------- */
static void analysis_1d(const double *in, int n, double *lo, double *hi,
                        const double *h, int L)
{
    for (int l = 0; l < n / 2; ++l) {
        double a = 0.0, d = 0.0;
        for (int k = 0; k < L; ++k) /* n - 2l = k, supp h = [0, L-1] */
            a += h[k] * in[pmod(2 * l + k, n)];
        for (int k = 2 - L; k <= 1; ++k) /* supp g = [2-L, 1] */
            d += gtap(h, L, k) * in[pmod(2 * l + k, n)];
        lo[l] = a;
        hi[l] = d;
    }
}

/* Inverse of analysis_1d: the expansion of Section 2.1,
 *     out[n] = sum_l h[n-2l] lo[l] + g[n-2l] hi[l],
 * written as the transpose (scatter) of the analysis sums. */
static void synthesis_1d(const double *lo, const double *hi, int n, double *out,
                         const double *h, int L)
{
    for (int i = 0; i < n; ++i) out[i] = 0.0;
    for (int l = 0; l < n / 2; ++l) {
        for (int k = 0; k < L; ++k)
            out[pmod(2 * l + k, n)] += h[k] * lo[l];
        for (int k = 2 - L; k <= 1; ++k)
            out[pmod(2 * l + k, n)] += gtap(h, L, k) * hi[l];
    }
}

/* ------------------------------------------------------------------------
 * 2-D separable isotropic transform (Section 2.2): at each scale the basis
 * functions are tensor products of 1-D scaling/wavelet functions of the SAME
 * scale, so each level transforms the current approximation band along x1
 * (every row) and then along x2 (every column), and recurses on the band that
 * is low-pass in both directions.  Forward transform Psi^* in place.
 * ---------------------------------------------------------------------- */
void or_fwt2(double *a, int n1, int n2, int levels, const double *h, int L)
{
    int nmax = n1 > n2 ? n1 : n2;
    double *t = (double *)malloc(sizeof(double) * nmax);
    double *lo = (double *)malloc(sizeof(double) * nmax);
    double *hi = (double *)malloc(sizeof(double) * nmax);
    int m1 = n1, m2 = n2;
    for (int lev = 1; lev <= levels; ++lev) {
        for (int r = 0; r < m2; ++r) { /* along x1 */
            for (int i = 0; i < m1; ++i) t[i] = a[r * n1 + i];
            analysis_1d(t, m1, lo, hi, h, L);
            for (int i = 0; i < m1 / 2; ++i) {
                a[r * n1 + i] = lo[i];
                a[r * n1 + m1 / 2 + i] = hi[i];
            }
        }
        for (int c = 0; c < m1; ++c) { /* along x2 */
            for (int i = 0; i < m2; ++i) t[i] = a[i * n1 + c];
            analysis_1d(t, m2, lo, hi, h, L);
            for (int i = 0; i < m2 / 2; ++i) {
                a[i * n1 + c] = lo[i];
                a[(m2 / 2 + i) * n1 + c] = hi[i];
            }
        }
        m1 /= 2;
        m2 /= 2;
    }
    free(t);
    free(lo);
    free(hi);
}

/* Inverse transform Psi (Section 2.2), in place: coarse to fine, each level
 * undoing the x2 step and then the x1 step. */
void or_ifwt2(double *a, int n1, int n2, int levels, const double *h, int L)
{
    int nmax = n1 > n2 ? n1 : n2;
    double *t = (double *)malloc(sizeof(double) * nmax);
    double *lo = (double *)malloc(sizeof(double) * nmax);
    double *hi = (double *)malloc(sizeof(double) * nmax);
    for (int lev = levels; lev >= 1; --lev) {
        int m1 = n1 >> (lev - 1), m2 = n2 >> (lev - 1);
        for (int c = 0; c < m1; ++c) { /* along x2 */
            for (int i = 0; i < m2 / 2; ++i) {
                lo[i] = a[i * n1 + c];
                hi[i] = a[(m2 / 2 + i) * n1 + c];
            }
            synthesis_1d(lo, hi, m2, t, h, L);
            for (int i = 0; i < m2; ++i) a[i * n1 + c] = t[i];
        }
        for (int r = 0; r < m2; ++r) { /* along x1 */
            for (int i = 0; i < m1 / 2; ++i) {
                lo[i] = a[r * n1 + i];
                hi[i] = a[r * n1 + m1 / 2 + i];
            }
            synthesis_1d(lo, hi, m1, t, h, L);
            for (int i = 0; i < m1; ++i) a[r * n1 + i] = t[i];
        }
    }
    free(t);
    free(lo);
    free(hi);
}

/* ------------------------------------------------------------------------
 * The blur operator as an integral operator (Section 1, eq. 1.1):
 *     (H f)(x) = sum_y K(x, y) f(y),   K(x, y) = S(x - y, y),
 * where S(., y) is the impulse response at source pixel y.  Operator 1 of
 * Section 4.1 uses isotropic Gaussian responses whose width depends on the
 * source row only; the caller passes that per-source-row 1-D profile k_y2 as
 * a table kt[y2][d + R], d in [-R, R], and the 2-D response is the outer
 * product S(d1, d2; y) = k_y2[d1] * k_y2[d2].
 *
 * H is evaluated as the plain gather over every source pixel y in the
 * (2R+1)^2 window that can reach x; H^T as the plain gather of the
 * transpose, (H^T r)(y) = sum_x K(x, y) r(x).  No separability is used.
 * ---------------------------------------------------------------------- */
void or_blur(const double *x, double *out, int n1, int n2, const double *kt,
             int R, int transpose)
{
    const int W = 2 * R + 1;
#pragma omp parallel for schedule(static)
    for (int o2 = 0; o2 < n2; ++o2) {
        for (int o1 = 0; o1 < n1; ++o1) {
            double acc = 0.0;
            for (int d2 = -R; d2 <= R; ++d2) {
                for (int d1 = -R; d1 <= R; ++d1) {
                    if (!transpose) {
                        /* source y = o - d, displacement d = o - y */
                        int y1 = pmod(o1 - d1, n1), y2 = pmod(o2 - d2, n2);
                        const double *k = kt + (size_t)y2 * W + R;
                        acc += k[d1] * k[d2] * x[y2 * n1 + y1];
                    } else {
                        /* output x = o + d reached from source o */
                        int x1 = pmod(o1 + d1, n1), x2 = pmod(o2 + d2, n2);
                        const double *k = kt + (size_t)o2 * W + R;
                        acc += k[d1] * k[d2] * x[x2 * n1 + x1];
                    }
                }
            }
            out[o2 * n1 + o1] = acc;
        }
    }
}

/* H applied to C planar channels; op_identity selects H = Id. */
static void apply_H(const double *x, double *out, int n1, int n2, int C,
                    const double *kt, int R, int op_identity, int transpose)
{
    size_t N = (size_t)n1 * n2;
    for (int c = 0; c < C; ++c) {
        if (op_identity)
            memcpy(out + c * N, x + c * N, sizeof(double) * N);
        else
            or_blur(x + c * N, out + c * N, n1, n2, kt, R, transpose);
    }
}

static void fwt_all(double *a, int n1, int n2, int C, int levels, const double *h, int L)
{
    size_t N = (size_t)n1 * n2;
    for (int c = 0; c < C; ++c) or_fwt2(a + c * N, n1, n2, levels, h, L);
}

static void ifwt_all(double *a, int n1, int n2, int C, int levels, const double *h, int L)
{
    size_t N = (size_t)n1 * n2;
    for (int c = 0; c < C; ++c) or_ifwt2(a + c * N, n1, n2, levels, h, L);
}

/* Gradient of the data term in the coefficient domain (Appendix A.1):
 *     grad(y) = Psi^* H^* (H Psi y - f0),
 * also returning r = H Psi y - f0 when r_out is not NULL. */
void or_grad(int n1, int n2, int C, int levels, const double *h, int L,
             const double *kt, int R, int op_identity, const double *f0,
             const double *y, double *grad, double *r_out)
{
    size_t NC = (size_t)n1 * n2 * C;
    double *x = (double *)malloc(sizeof(double) * NC);
    double *r = (double *)malloc(sizeof(double) * NC);
    memcpy(x, y, sizeof(double) * NC);
    ifwt_all(x, n1, n2, C, levels, h, L);                 /* x = Psi y      */
    apply_H(x, r, n1, n2, C, kt, R, op_identity, 0);      /* r = H x        */
    for (size_t i = 0; i < NC; ++i) r[i] -= f0[i];        /* r = H x - f0   */
    apply_H(r, grad, n1, n2, C, kt, R, op_identity, 1);   /* s = H^T r      */
    fwt_all(grad, n1, n2, C, levels, h, L);               /* g = Psi^* s    */
    if (r_out) memcpy(r_out, r, sizeof(double) * NC);
    free(x);
    free(r);
}

/* Proximal operator of the weighted l1 norm of Section 4.3 (eq. 4.1),
 * ||z||_{1,w} = sum w[l] |z[l]|, scaled by the step t:  soft thresholding
 * z = sign(v) max(|v| - t w, 0).  Joint mode (an extension for colour
 * images, not in the paper): group soft thresholding of the C channel values
 * of each coefficient, z_c = v_c max(0, 1 - t w / ||v||_2), using the weight
 * of channel 0. */
static void prox(const double *v, double *z, size_t N, int C, const double *w,
                 double t, int joint)
{
    if (!joint) {
        for (size_t i = 0; i < N * C; ++i) {
            double a = fabs(v[i]) - t * w[i];
            z[i] = a > 0.0 ? (v[i] > 0.0 ? a : -a) : 0.0;
        }
        return;
    }
    for (size_t i = 0; i < N; ++i) {
        double nrm2 = 0.0;
        for (int c = 0; c < C; ++c) nrm2 += v[c * N + i] * v[c * N + i];
        double nrm = sqrt(nrm2);
        double s = nrm > 0.0 ? 1.0 - t * w[i] / nrm : 0.0;
        if (s < 0.0) s = 0.0;
        for (int c = 0; c < C; ++c) z[c * N + i] = v[c * N + i] * s;
    }
}

/* Weighted l1 norm (Section 4.3); joint mode uses the channel l2 norm. */
static double wl1(const double *z, size_t N, int C, const double *w, int joint)
{
    double s = 0.0;
    if (!joint) {
        for (size_t i = 0; i < N * C; ++i) s += w[i] * fabs(z[i]);
        return s;
    }
    for (size_t i = 0; i < N; ++i) {
        double nrm2 = 0.0;
        for (int c = 0; c < C; ++c) nrm2 += z[c * N + i] * z[c * N + i];
        s += w[i] * sqrt(nrm2);
    }
    return s;
}

/* Energy of eq. 4.1 evaluated at f = Psi z:  1/2 ||H Psi z - f0||^2 +
 * ||z||_{1,w}.  Writes the two terms to terms[0], terms[1] if non-NULL. */
double or_energy(int n1, int n2, int C, int levels, const double *h, int L,
                 const double *kt, int R, int op_identity, const double *w,
                 int joint, const double *f0, const double *z, double *terms)
{
    size_t N = (size_t)n1 * n2, NC = N * C;
    double *x = (double *)malloc(sizeof(double) * NC);
    double *r = (double *)malloc(sizeof(double) * NC);
    memcpy(x, z, sizeof(double) * NC);
    ifwt_all(x, n1, n2, C, levels, h, L);
    apply_H(x, r, n1, n2, C, kt, R, op_identity, 0);
    double d = 0.0;
    for (size_t i = 0; i < NC; ++i) d += 0.5 * (r[i] - f0[i]) * (r[i] - f0[i]);
    double g = wl1(z, N, C, w, joint);
    if (terms) {
        terms[0] = d;
        terms[1] = g;
    }
    free(x);
    free(r);
    return d + g;
}

/* ------------------------------------------------------------------------
 * FISTA / forward-backward for the coefficient form of eq. 4.1
 * (Appendix A.1, eq. A.1), starting from z^(0) = y^(1) = init and, for
 * i = 1 .. iters,
 *     z^(i)   = Prox_{tau ||.||_{1,w}} ( y^(i) - tau grad(y^(i)) )
 *     y^(i+1) = z^(i) + (i-1)/(i+2) (z^(i) - z^(i-1)).
 * init == NULL selects init = Psi^* f0.  Outputs z^(iters) in z_out (may be
 * NULL) and f = Psi z^(iters) in f_out (may be NULL).
 *
 * log (may be NULL) receives 3 doubles per iteration i:
 *   [1/2 ||H Psi y^(i) - f0||^2, ||y^(i)||_{1,w}, ||z^(i) - y^(i)||^2].
 * tape (may be NULL) receives v^(i) = y^(i) - tau grad(y^(i)), the argument of
 * the prox at iteration i, as iters consecutive C*n1*n2 blocks.
 * ---------------------------------------------------------------------- */
int or_fista(int n1, int n2, int C, int levels, const double *h, int L,
             const double *kt, int R, int op_identity, const double *w,
             int joint, double tau, int iters, const double *f0,
             const double *init, double *z_out, double *f_out, double *log,
             double *tape)
{
    size_t N = (size_t)n1 * n2, NC = N * C;
    double *y = (double *)malloc(sizeof(double) * NC);
    double *z = (double *)malloc(sizeof(double) * NC);
    double *zprev = (double *)malloc(sizeof(double) * NC);
    double *g = (double *)malloc(sizeof(double) * NC);
    double *r = (double *)malloc(sizeof(double) * NC);
    double *v = (double *)malloc(sizeof(double) * NC);
    if (init) {
        memcpy(y, init, sizeof(double) * NC);
    } else {
        memcpy(y, f0, sizeof(double) * NC);
        fwt_all(y, n1, n2, C, levels, h, L);
    }
    memcpy(zprev, y, sizeof(double) * NC); /* z^(0) = y^(1) */
    memcpy(z, y, sizeof(double) * NC);     /* z^(0) when iters == 0 */
    for (int i = 1; i <= iters; ++i) {
        or_grad(n1, n2, C, levels, h, L, kt, R, op_identity, f0, y, g, r);
        for (size_t k = 0; k < NC; ++k) v[k] = y[k] - tau * g[k];
        prox(v, z, N, C, w, tau, joint);
        if (log) {
            double dt = 0.0, gm = 0.0;
            for (size_t k = 0; k < NC; ++k) {
                dt += 0.5 * r[k] * r[k];
                gm += (z[k] - y[k]) * (z[k] - y[k]);
            }
            log[3 * (i - 1) + 0] = dt;
            log[3 * (i - 1) + 1] = wl1(y, N, C, w, joint);
            log[3 * (i - 1) + 2] = gm;
        }
        if (tape) memcpy(tape + (size_t)(i - 1) * NC, v, sizeof(double) * NC);
        double beta = (double)(i - 1) / (double)(i + 2);
        for (size_t k = 0; k < NC; ++k) {
            y[k] = z[k] + beta * (z[k] - zprev[k]);
            zprev[k] = z[k];
        }
    }
    if (z_out) memcpy(z_out, z, sizeof(double) * NC);
    if (f_out) {
        memcpy(f_out, z, sizeof(double) * NC);
        ifwt_all(f_out, n1, n2, C, levels, h, L);
    }
    free(y);
    free(z);
    free(zprev);
    free(g);
    free(r);
    free(v);
    return 0;
}

/* ------------------------------------------------------------------------
 * Reverse mode of or_fista with init = Psi^* f0 and the scalar (non-joint)
 * prox, on the full tape of prox arguments v^(i).  Given fbar = dLoss/df for
 * f = Psi z^(K), returns dLoss/df0 in f0bar and dLoss/dw in wbar (either may
 * be NULL).  Derivation (chain rule through the recursion above):
 *   zbar^(K) = Psi^* fbar
 *   y^(i+1) = (1+b_i) z^(i) - b_i z^(i-1)   ->  zbar^(i) += (1+b_i) ybar^(i+1),
 *                                              zbar^(i-1) -= b_i ybar^(i+1)
 *   z^(i) = S_{tau w}(v^(i))               ->  vbar = zbar^(i) 1{|v| > tau w},
 *                                              wbar -= tau zbar^(i) sign(v) 1{|v| > tau w}
 *   v^(i) = y^(i) - tau A^T (A y^(i) - f0), A = H Psi
 *                                          ->  ybar^(i) = vbar - tau A^T A vbar,
 *                                              f0bar  += tau A vbar
 *   y^(1) = z^(0) = Psi^* f0               ->  f0bar  += Psi ybar^(1)
 * with b_i = (i-1)/(i+2); the kink |v| = tau w gets derivative 0.
 * ---------------------------------------------------------------------- */
int or_fista_reverse(int n1, int n2, int C, int levels, const double *h, int L,
                     const double *kt, int R, int op_identity, const double *w,
                     double tau, int iters, const double *tape,
                     const double *fbar, double *f0bar, double *wbar)
{
    size_t NC = (size_t)n1 * n2 * C;
    double *zb = (double *)calloc(NC, sizeof(double));  /* zbar^(i)           */
    double *zbm = (double *)calloc(NC, sizeof(double)); /* partial zbar^(i-1) */
    double *yb = (double *)calloc(NC, sizeof(double));
    double *vb = (double *)calloc(NC, sizeof(double));
    double *x = (double *)malloc(sizeof(double) * NC);
    double *q = (double *)malloc(sizeof(double) * NC);
    double *s = (double *)malloc(sizeof(double) * NC);
    double *fb0 = (double *)calloc(NC, sizeof(double));
    double *wb = (double *)calloc(NC, sizeof(double));

    memcpy(zb, fbar, sizeof(double) * NC);
    fwt_all(zb, n1, n2, C, levels, h, L); /* zbar^(K) = Psi^* fbar */
    for (int i = iters; i >= 1; --i) {
        const double *v = tape + (size_t)(i - 1) * NC;
        for (size_t k = 0; k < NC; ++k) {
            int act = fabs(v[k]) > tau * w[k];
            vb[k] = act ? zb[k] : 0.0;
            if (act) wb[k] -= tau * zb[k] * (v[k] > 0.0 ? 1.0 : -1.0);
        }
        /* ybar^(i) = vbar - tau Psi^* H^T H Psi vbar ; f0bar += tau H Psi vbar */
        memcpy(x, vb, sizeof(double) * NC);
        ifwt_all(x, n1, n2, C, levels, h, L);
        apply_H(x, q, n1, n2, C, kt, R, op_identity, 0);
        for (size_t k = 0; k < NC; ++k) fb0[k] += tau * q[k];
        apply_H(q, s, n1, n2, C, kt, R, op_identity, 1);
        fwt_all(s, n1, n2, C, levels, h, L);
        for (size_t k = 0; k < NC; ++k) yb[k] = vb[k] - tau * s[k];
        if (i >= 2) {
            /* y^(i) = (1+b) z^(i-1) - b z^(i-2), b = b_{i-1} */
            double b = (double)(i - 2) / (double)(i + 1);
            for (size_t k = 0; k < NC; ++k) {
                zb[k] = zbm[k] + (1.0 + b) * yb[k]; /* now complete zbar^(i-1) */
                zbm[k] = -b * yb[k];                /* partial zbar^(i-2)     */
            }
        }
    }
    /* y^(1) = z^(0) = Psi^* f0: zbar^(0) = zbm (zero, since b_1 = 0) + ybar^(1) */
    if (iters >= 1) {
        for (size_t k = 0; k < NC; ++k) x[k] = yb[k] + zbm[k];
    } else {
        memcpy(x, zb, sizeof(double) * NC);
    }
    ifwt_all(x, n1, n2, C, levels, h, L);
    for (size_t k = 0; k < NC; ++k) fb0[k] += x[k];
    if (f0bar) memcpy(f0bar, fb0, sizeof(double) * NC);
    if (wbar) memcpy(wbar, wb, sizeof(double) * NC);
    free(zb);
    free(zbm);
    free(yb);
    free(vb);
    free(x);
    free(q);
    free(s);
    free(fb0);
    free(wb);
    return 0;
}
