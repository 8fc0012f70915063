// pd_decomp.h -- kernels of Algorithm 1 (Section 3.2, Algorithm 1; Section 5):
// the wavelet representation Theta~ = sum_k A~_k B_k of a product-convolution
// operator, in FP64.  Internal to libpd.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pd {

// A wavelet sub-band of an n1 x n2 Mallat plane: level (1 finest), origin and grid.
struct DecBand {
    int lev, o2, o1, g2, g1;
};

// One kept entry of a circulant generator: band-grid position and value.
struct DecEntry {
    int q2, q1;
    double val;
};

// Kept generators of all terms.  Pair p = (k nb + b') nb + b (source band b', target band b):
// entries ent[off[p] .. off[p] + cnt[p]); for a coarser target (lev_b > lev_b') they are grouped
// by the residue (q2 mod f, q1 mod f), f = 2^(lev_b - lev_b'), with class r in
// [res[roff[p] + r], res[roff[p] + r + 1]) relative to off[p].
struct DecTables {
    const DecBand *bands;  // [nb]
    const int64_t *off;    // [m nb nb]
    const int *cnt;        // [m nb nb]
    const int64_t *roff;   // [m nb nb]
    const int *res;        // residue offsets
    const DecEntry *ent;
    int nb, n1, n2;
};

// planes[p] = e_{base + p} (a Dirac at Mallat position base + p; a zero plane past N), p < P
hipError_t launch_dec_dirac(double *planes, int64_t base, int P, int64_t N, hipStream_t s);
// planes[p] = e_{pos[p]} for the positions pos (device), p < P
hipError_t launch_dec_dirac_at(double *planes, const int *pos, int P, int64_t N, hipStream_t s);
// out[p] = u * in[p] (periodic convolution, transpose = 0) or the correlation (transpose = 1)
hipError_t launch_dec_conv(const double *in, double *out, int P, const double *u, int R, int n1, int n2,
                           int transpose, hipStream_t s);
// out[p] = v . in[p]
hipError_t launch_dec_mul(const double *in, const double *v, double *out, int P, int64_t N, hipStream_t s);
// acc[j] += A~_k y[j] for the P columns y[j] (one workgroup per column), term k
hipError_t launch_dec_acc(const double *y, double *acc, int P, const DecTables &t, int k, hipStream_t s);
// cnt[j] = number of nonzero entries of acc[j]
hipError_t launch_dec_count(const double *acc, int P, int64_t N, int64_t *cnt, hipStream_t s);
// rows / vals from base[j] on: the nonzero entries of acc[j] in row order
hipError_t launch_dec_fill(const double *acc, int P, int64_t N, const int64_t *base, int *rows, double *vals,
                           hipStream_t s);

}  // namespace pd
