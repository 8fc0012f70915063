/* Runs every exported oracle routine once on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Inputs: argv[1] = a text
 * file holding the low-pass filter length and its taps, argv[2] = a text file
 * holding R and the (2R+1)-tap profile of every row (n2 rows).  Prints OK. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void or_fwt2(double *a, int n1, int n2, int levels, const double *h, int L);
void or_ifwt2(double *a, int n1, int n2, int levels, const double *h, int L);
void or_blur(const double *x, double *out, int n1, int n2, const double *kt, int R, int transpose);
void or_grad(int n1, int n2, int C, int levels, const double *h, int L, const double *kt, int R,
             int op_identity, const double *f0, const double *y, double *g, double *r_out);
double or_energy(int n1, int n2, int C, int levels, const double *h, int L, const double *kt, int R,
                 int op_identity, const double *w, int joint, const double *f0, const double *z,
                 double *terms);
int or_fista(int n1, int n2, int C, int levels, const double *h, int L, const double *kt, int R,
             int op_identity, const double *w, int joint, double tau, int iters, const double *f0,
             const double *init, double *z_out, double *f_out, double *log, double *tape);
int or_fista_reverse(int n1, int n2, int C, int levels, const double *h, int L, const double *kt, int R,
                     int op_identity, const double *w, double tau, int iters, const double *tape,
                     const double *fbar, double *f0bar, double *wbar);

static int finite_all(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int main(int argc, char **argv)
{
    if (argc < 3) return 2;
    FILE *fh = fopen(argv[1], "r"), *fk = fopen(argv[2], "r");
    if (!fh || !fk) return 2;
    int L = 0, R = 0;
    if (fscanf(fh, "%d", &L) != 1 || L < 2 || L > 20) return 2;
    double h[20];
    for (int k = 0; k < L; ++k)
        if (fscanf(fh, "%lf", &h[k]) != 1) return 2;
    const int n1 = 24, n2 = 16, C = 2, levels = 3, iters = 6;
    if (fscanf(fk, "%d", &R) != 1 || R < 0 || R > 9) return 2;
    const int W = 2 * R + 1;
    double *kt = malloc(sizeof(double) * n2 * W);
    for (int i = 0; i < n2 * W; ++i)
        if (fscanf(fk, "%lf", &kt[i]) != 1) return 2;
    fclose(fh);
    fclose(fk);
    const size_t N = (size_t)n1 * n2, NC = N * C;
    double *a = malloc(sizeof(double) * NC), *b = malloc(sizeof(double) * NC);  /* (b: NC for or_grad's r) */
    double *f0 = malloc(sizeof(double) * NC), *w = malloc(sizeof(double) * NC);
    double *z = malloc(sizeof(double) * NC), *f = malloc(sizeof(double) * NC);
    double *g = malloc(sizeof(double) * NC), *log = malloc(sizeof(double) * 3 * iters);
    double *tape = malloc(sizeof(double) * NC * iters);
    double *f0b = malloc(sizeof(double) * NC), *wb = malloc(sizeof(double) * NC);
    unsigned s = 12345u;
    for (size_t i = 0; i < NC; ++i) {
        s = s * 1103515245u + 12345u;
        f0[i] = (double)(s >> 8) / (double)(1u << 24) - 0.5;
        w[i] = 0.02 + 0.01 * (double)(i % 7);
    }
    /* transforms: round trip */
    memcpy(a, f0, sizeof(double) * N);
    or_fwt2(a, n1, n2, levels, h, L);
    or_ifwt2(a, n1, n2, levels, h, L);
    double err = 0.0;
    for (size_t i = 0; i < N; ++i) err = fmax(err, fabs(a[i] - f0[i]));
    if (err > 1e-9) { printf("fwt round trip %g\n", err); return 1; }
    /* operator and its transpose */
    or_blur(f0, a, n1, n2, kt, R, 0);
    or_blur(f0, b, n1, n2, kt, R, 1);
    if (!finite_all(a, N) || !finite_all(b, N)) return 1;
    /* gradient, energy (scalar and joint), forward and reverse solves */
    double terms[2];
    or_grad(n1, n2, C, levels, h, L, kt, R, 0, f0, f0, g, b);
    or_grad(n1, n2, C, levels, h, L, kt, R, 1, f0, f0, g, NULL);
    (void)or_energy(n1, n2, C, levels, h, L, kt, R, 0, w, 0, f0, g, terms);
    (void)or_energy(n1, n2, C, levels, h, L, kt, R, 0, w, 1, f0, g, terms);
    for (int joint = 0; joint < 2; ++joint)
        if (or_fista(n1, n2, C, levels, h, L, kt, R, 0, w, joint, 0.5, iters, f0, NULL, z, f, log, tape)) return 1;
    if (or_fista(n1, n2, C, levels, h, L, kt, R, 1, w, 0, 0.5, iters, f0, z, z, f, NULL, NULL)) return 1;
    if (or_fista(n1, n2, C, levels, h, L, kt, R, 0, w, 0, 0.5, iters, f0, NULL, z, f, log, tape)) return 1;
    if (or_fista_reverse(n1, n2, C, levels, h, L, kt, R, 0, w, 0.5, iters, tape, f, f0b, wb)) return 1;
    if (!finite_all(f, NC) || !finite_all(f0b, NC) || !finite_all(wb, NC) || !finite_all(log, 3 * iters)) return 1;
    free(kt); free(a); free(b); free(f0); free(w); free(z); free(f); free(g); free(log); free(tape);
    free(f0b); free(wb);
    printf("OK\n");
    return 0;
}
