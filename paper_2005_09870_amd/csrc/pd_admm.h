// pd_admm.h -- kernels of ADMM with a product-convolution operator (ADMM-PC,
// Appendix A.2; Table 1): a radix-2 2-D FFT for power-of-two sizes and the
// element-wise steps of the iteration.  Internal to libpd.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pd_kernels.h"

namespace pd {

template <typename T>
struct Cx {
    T re, im;
};

// In-place 2-D FFT of `batch` planes n2 x n1 (interleaved complex, row-major):
// rows then columns, radix-2 Stockham autosort in LDS.  tw1 / tw2: tables
// exp(-2 pi i t / n), t < n/2, for n1 and n2.  inverse: conjugate twiddles and
// a 1/(n1 n2) scale.  n1, n2 powers of two >= 2 with 2 n sizeof(Cx<T>) <= 64 KiB
// (4096 in FP32, 2048 in FP64).
template <typename T>
hipError_t launch_fft2(Cx<T> *data, int n1, int n2, int batch, const Cx<T> *tw1, const Cx<T> *tw2, int inverse,
                       hipStream_t s);

// One pass of launch_fft2: rows (cols == 0, table tw1) or columns (cols != 0, table tw2, with the
// inverse's scale).
template <typename T>
hipError_t launch_fft_pass(Cx<T> *data, int n1, int n2, int batch, const Cx<T> *tw, int inverse, int cols,
                           hipStream_t s);

// Element-wise steps (N pixels, m terms, plane stride N).
template <typename T>
struct AdmmArgs {
    int n1, n2, m, levels;
    int64_t N;
    T beta1, beta2;
    const T *gam;           // device [m]: gamma_k
    const T *v;             // [m][N] multipliers
    const Cx<T> *uh;        // [m][N] kernel spectra
    const T *mh;            // [N]: 1 + sum_k |u_k^|^2 / (beta1 gamma_k)
    const T *den;           // [N]: beta1 sum_k gamma_k v_k^2 + beta2
    const T *utf0;          // [m][N]: U_k^T f0
    T *g, *xi;              // [m][N]; g holds a_k between the a-step and the g-step
    T *f, *z, *zeta;        // [N]
    T *tz;                  // [N]: Psi^* f
    T *tf;                  // [N]: beta2 z + zeta (then Psi of it, in tfs)
    const T *tfs;           // [N]: Psi (beta2 z + zeta)
    Cx<T> *cb;              // [m][N] complex planes of the g-step
    const T *wmap;          // per-coefficient weights or nullptr (then wlev by band)
    T wlev[PD_MAXL + 1];
    double *slots;          // this iteration's [3][PD_NSLOT] (nullptr: off): ||g - V f||_D^2,
                            // ||z - Psi^* f||^2, ||z||_{1,w}
    double *slots_next;     // the next iteration's (row 2, written with its z), or nullptr
};

// a_k = (U_k^T f0 - xi_k) / (beta1 gamma_k) + v_k f into g_k and cb_k (imaginary 0), all k
template <typename T> hipError_t launch_admm_a(const AdmmArgs<T> &a, hipStream_t s);
// per frequency: q = sum_k u_k^ cb_k / mh; cb_k = conj(u_k^) q, all k
template <typename T> hipError_t launch_admm_accq(const AdmmArgs<T> &a, hipStream_t s);
// z = soft(tz - zeta/beta2, w/beta2); tf = beta2 z + zeta; slots row 2 += w |z|
template <typename T> hipError_t launch_admm_z(const AdmmArgs<T> &a, hipStream_t s);
// g_k = a_k - Re(cb_k) / (beta1 gamma_k); f = (sum_k v_k (xi_k + beta1 gamma_k g_k) + tfs) / den;
// xi_k += beta1 gamma_k (g_k - v_k f) (slots row 0); with `next`, the next a_k into g_k and cb_k
template <typename T> hipError_t launch_admm_f(const AdmmArgs<T> &a, int next, hipStream_t s);
// zeta += beta2 (z - tz) (slots row 1); with `next`, the next z and tf as launch_admm_z (slots_next row 2)
template <typename T> hipError_t launch_admm_zeta(const AdmmArgs<T> &a, int next, hipStream_t s);

// Set-up: u_k placed at offsets (d mod n) into cb-like planes [m][N] (complex, imaginary 0)
template <typename T>
hipError_t launch_admm_padk(const T *u, int R, int m, int n1, int n2, Cx<T> *out, hipStream_t s);
// mx[k] = max |u_k^| (one workgroup per k)
template <typename T> hipError_t launch_admm_absmax(const Cx<T> *uh, int m, int64_t N, T *mx, hipStream_t s);
// gam[k] = mx[k] / sum_j mx[j] (1/m if the sum is 0); m <= 64
template <typename T> hipError_t launch_admm_gamma(const T *mx, int m, T *gam, hipStream_t s);
// tw[t] = exp(-2 pi i t / n) for t < n/2
template <typename T> hipError_t launch_admm_twiddle(Cx<T> *tw, int n, hipStream_t s);
// mh, den from gamma (device), uh, v
template <typename T> hipError_t launch_admm_diag(const AdmmArgs<T> &a, hipStream_t s);
// out_k = conj(u_k^) * fh for all k (for U_k^T f0), then after an inverse FFT: out = Re(x)
template <typename T> hipError_t launch_admm_conjmul(const Cx<T> *uh, const Cx<T> *fh, Cx<T> *out, int m,
                                                     int64_t N, hipStream_t s);
template <typename T> hipError_t launch_admm_real(const T *x, Cx<T> *out, int64_t N, hipStream_t s);
template <typename T> hipError_t launch_admm_takere(const Cx<T> *x, T *out, int64_t n, hipStream_t s);

}  // namespace pd
