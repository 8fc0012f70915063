// pd_wkernels.h -- argument blocks and launchers of the gfx950 kernels of
// FISTA in the wavelet domain (FISTA-W / FISTA-WP, Section 4.3 and Appendix
// A.1): products with the sparse matrix Theta_L and its transpose, the fused
// (preconditioned) prox + momentum, the Jacobi diagonal and a CSR transpose.
// Internal to libpd; the public interface is include/pd.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pd_kernels.h"

namespace pd {

// A CSR matrix as the kernels read it.  Row bounds are clamped to [0, nnz]
// and column indices to [0, ncol) on the fly, so malformed input gives
// meaningless numbers but no access outside the arrays.
template <typename T>
struct Csr {
    const int64_t *rp;      // [n + 1]
    const int32_t *col;     // [nnz]
    const T *val;           // [nnz]
    int n;                  // rows (= columns here)
    int64_t nnz;
};

// u = A x - b (b may be nullptr); slots (nullptr: off) receives 1/2 ||u||^2 in row 0.
template <typename T>
struct WResArgs {
    Csr<T> a;
    const T *x, *b;
    T *u;
    double *slots;
};

// One FISTA-W(P) update per row l of At = Theta_L^T:
//   g = (At u)_l, v = y_l - tau s_l g, z = soft(v, tau s_l w_l),
//   zn_l = z, y_l <- z + beta_next (z - zc_l)
// with s_l = sigma[l] (nullptr: 1).  slots rows 1, 2: sum w |y|, sum (z - y)^2.
template <typename T>
struct WProxArgs {
    Csr<T> at;
    const T *u;
    T *y;                   // y(i) in, y(i+1) out
    const T *zc;            // z(i-1)
    T *zn;                  // z(i) out (the z(i-2) plane)
    const T *sigma;         // Jacobi preconditioner or nullptr
    const T *wmap;          // per-coefficient weights or nullptr (then wlev by band)
    T wlev[PD_MAXL + 1];
    int n1, n2, levels;     // Mallat plane of the coefficients (band of a row)
    T tau, beta_next;
    double *slots;
    int *flag;              // set to 1 if v is not finite
};

// Threads of a row group for an average row length (a power of two, 4..32).
int wgroup_for(int64_t nnz, int n);

template <typename T> hipError_t launch_wres(const WResArgs<T> &a, int group, hipStream_t s);
template <typename T> hipError_t launch_wprox(const WProxArgs<T> &a, int group, hipStream_t s);
// sigma[l] = 1 / sum_k At[l, k]^2, or 1 for an empty row of At (column of Theta_L)
template <typename T> hipError_t launch_wjacobi(const Csr<T> &at, T *sigma, int group, hipStream_t s);
// y = zc + beta (zc - zp)
template <typename T> hipError_t launch_wform_y(const T *zc, const T *zp, T beta, T *y, int64_t n, hipStream_t s);

// CSR transpose (set-up): check, count, scan, scatter, per-row sort.
hipError_t launch_csr_check(const int64_t *rp, const int32_t *col, int n, int64_t nnz, int *flag, hipStream_t s);
hipError_t launch_fill_i32(int *p, int v, int64_t n, hipStream_t s);
hipError_t launch_csr_count(const int64_t *rp, const int32_t *col, int n, int *cnt, hipStream_t s);
hipError_t launch_csr_scan(const int *cnt, int n, int64_t *trp, hipStream_t s);
template <typename T>
hipError_t launch_csr_scatter(const Csr<T> &a, const int64_t *trp, int *cur, int32_t *tcol, T *tval, hipStream_t s);
template <typename T>
hipError_t launch_csr_sort(const int64_t *trp, int n, int32_t *tcol, T *tval, hipStream_t s);

}  // namespace pd
