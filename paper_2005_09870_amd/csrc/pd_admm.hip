// pd_admm.hip -- gfx950 kernels of ADMM-PC (Appendix A.2; Table 1).
//
// The g-subproblem (U^T U + beta1 D) g = rhs is solved with the Woodbury
// identity, whose middle matrix Id + sum_k U_k U_k^T / (beta1 gamma_k) is
// diagonal in the Fourier basis: a radix-2 2-D FFT (rows, then blocks of
// columns, each a Stockham autosort in LDS) and element-wise products.  The
// other steps (prox, f-update, multiplier updates) are element-wise passes;
// the wavelet transforms are the solver's own kernels.
#include <hip/hip_runtime.h>

#include "pd_admm.h"

namespace pd {

namespace {

constexpr int NTF = 256;

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b)
{
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// n-point FFTs of `cnt` sequences held in LDS at A[c * n + i] (ping-pong with B),
// log2n stages of radix-2 Stockham; returns the buffer holding the result.
template <typename T>
__device__ Cx<T> *stockham(Cx<T> *A, Cx<T> *B, int n, int log2n, int cnt, const Cx<T> *__restrict__ tw, bool inverse)
{
    const int half = n >> 1;
    for (int s = 0; s < log2n; ++s) {
        const int m = 1 << s;
        for (int j = threadIdx.x; j < cnt * half; j += NTF) {
            const int c = j >> (log2n - 1), jj = j & (half - 1);
            const int k = jj & (m - 1), g = jj >> s;
            Cx<T> w = tw[k << (log2n - 1 - s)];  // exp(-+2 pi i k / (2m))
            if (inverse) w.im = -w.im;
            const Cx<T> a = A[c * n + g * m + k], b = A[c * n + g * m + k + half];
            const Cx<T> wb = cmul(w, b);
            B[c * n + 2 * g * m + k] = Cx<T>{a.re + wb.re, a.im + wb.im};
            B[c * n + 2 * g * m + k + m] = Cx<T>{a.re - wb.re, a.im - wb.im};
        }
        __syncthreads();
        Cx<T> *t = A;
        A = B;
        B = t;
    }
    return A;
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_fft_rows(Cx<T> *data, int n1, int log2n1, const Cx<T> *tw, int inverse)
{
    extern __shared__ unsigned char lds_raw[];
    Cx<T> *A = reinterpret_cast<Cx<T> *>(lds_raw);
    Cx<T> *B = A + n1;
    Cx<T> *row = data + (int64_t)blockIdx.x * n1;
    for (int i = threadIdx.x; i < n1; i += NTF) A[i] = row[i];
    __syncthreads();
    Cx<T> *R = stockham<T>(A, B, n1, log2n1, 1, tw, inverse != 0);
    for (int i = threadIdx.x; i < n1; i += NTF) row[i] = R[i];
}

// cb consecutive columns of one plane per workgroup (grid: (n1 / cb, batch)).
template <typename T>
__global__ __launch_bounds__(NTF) void k_fft_cols(Cx<T> *data, int n1, int n2, int log2n2, int cb, const Cx<T> *tw,
                                                  int inverse, T scale)
{
    extern __shared__ unsigned char lds_raw[];
    Cx<T> *A = reinterpret_cast<Cx<T> *>(lds_raw);
    Cx<T> *B = A + cb * n2;
    Cx<T> *plane = data + (int64_t)blockIdx.y * n1 * n2;
    const int c0 = blockIdx.x * cb;
    for (int e = threadIdx.x; e < cb * n2; e += NTF) {  // lane-contiguous along the row: coalesced
        const int r = e / cb, c = e - r * cb;
        A[c * n2 + r] = plane[(int64_t)r * n1 + c0 + c];
    }
    __syncthreads();
    Cx<T> *R = stockham<T>(A, B, n2, log2n2, cb, tw, inverse != 0);
    for (int e = threadIdx.x; e < cb * n2; e += NTF) {
        const int r = e / cb, c = e - r * cb;
        const Cx<T> v = R[c * n2 + r];
        plane[(int64_t)r * n1 + c0 + c] = Cx<T>{v.re * scale, v.im * scale};
    }
}

inline int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

__device__ __forceinline__ int band_of(int i1, int i2, int n1, int n2, int L)
{
    int t1 = L, t2 = L;
    while (t1 > 0 && i1 >= (n1 >> t1)) --t1;
    while (t2 > 0 && i2 >= (n2 >> t2)) --t2;
    const int t = t1 < t2 ? t1 : t2;
    return t == L ? 0 : L - t;
}

template <int NV>
__device__ void slots_add(double (&v)[NV], double *slots)
{
    __shared__ double red[NV][NTF / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double a = v[q];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) a += __shfl_xor(a, m);
        if (lane == 0) red[q][wv] = a;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < NTF / 64; ++w) a += red[threadIdx.x][w];
        atomicAdd(slots + threadIdx.x * PD_NSLOT + (blockIdx.x % PD_NSLOT), a);
    }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + NTF - 1) / NTF); }

template <typename T>
__global__ void k_admm_a(AdmmArgs<T> a, int k)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    const T bg = a.beta1 * a.gam[k];
    const int64_t o = (int64_t)k * a.N + i;
    const T ak = (a.utf0[o] - a.xi[o] + bg * a.v[o] * a.f[i]) / bg;
    a.g[o] = ak;
    a.cb[i] = Cx<T>{ak, T(0)};
}

template <typename T>
__global__ void k_admm_acc(AdmmArgs<T> a, int k)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    const Cx<T> p = cmul(a.uh[(int64_t)k * a.N + i], a.cb[i]);
    if (k == 0) {
        a.th[i] = p;
    } else {
        const Cx<T> t = a.th[i];
        a.th[i] = Cx<T>{t.re + p.re, t.im + p.im};
    }
}

template <typename T>
__global__ void k_admm_q(AdmmArgs<T> a, int k)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    Cx<T> u = a.uh[(int64_t)k * a.N + i];
    u.im = -u.im;
    const T im = T(1) / a.mh[i];
    const Cx<T> t = a.th[i];
    a.cb[i] = cmul(u, Cx<T>{t.re * im, t.im * im});
}

template <typename T>
__global__ void k_admm_g(AdmmArgs<T> a, int k)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    const int64_t o = (int64_t)k * a.N + i;
    a.g[o] -= a.cb[i].re / (a.beta1 * a.gam[k]);
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_z(AdmmArgs<T> a)
{
    __shared__ T sw[PD_MAXL + 1];
    if (!a.wmap && threadIdx.x <= a.levels) sw[threadIdx.x] = a.wlev[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    double st[1] = {0.0};
    if (i < a.N) {
        T w;
        if (a.wmap) {
            w = a.wmap[i];
        } else {
            const int i2 = (int)(i / a.n1), i1 = (int)(i - (int64_t)i2 * a.n1);
            w = sw[band_of(i1, i2, a.n1, a.n2, a.levels)];
        }
        const T v = a.tz[i] - a.zeta[i] / a.beta2;
        const T t = w / a.beta2;
        const T m = fabs(v) - t;
        const T z = m > T(0) ? copysign(m, v) : T(0);
        a.z[i] = z;
        a.tf[i] = a.beta2 * z + a.zeta[i];
        st[0] = (double)w * fabs((double)z);
    }
    if (a.slots) slots_add<1>(st, a.slots + 2 * PD_NSLOT);
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_f(AdmmArgs<T> a)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    double st[1] = {0.0};
    if (i < a.N) {
        T acc = a.tf[i];
        for (int k = 0; k < a.m; ++k) {
            const int64_t o = (int64_t)k * a.N + i;
            acc += a.v[o] * (a.xi[o] + a.beta1 * a.gam[k] * a.g[o]);
        }
        const T f = acc / a.den[i];
        a.f[i] = f;
        for (int k = 0; k < a.m; ++k) {
            const int64_t o = (int64_t)k * a.N + i;
            const T r = a.g[o] - a.v[o] * f;
            a.xi[o] += a.beta1 * a.gam[k] * r;
            st[0] += (double)a.gam[k] * (double)r * (double)r;
        }
    }
    if (a.slots) slots_add<1>(st, a.slots);
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_zeta(AdmmArgs<T> a)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    double st[1] = {0.0};
    if (i < a.N) {
        const T r = a.z[i] - a.tz[i];
        a.zeta[i] += a.beta2 * r;
        st[0] = (double)r * (double)r;
    }
    if (a.slots) slots_add<1>(st, a.slots + PD_NSLOT);
}

template <typename T>
__global__ void k_admm_padk(const T *u, int R, int m, int n1, int n2, Cx<T> *out)
{
    const int64_t N = (int64_t)n1 * n2;
    const int64_t e = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (e >= (int64_t)m * N) return;
    const int k = (int)(e / N);
    const int64_t p = e - (int64_t)k * N;
    const int i2 = (int)(p / n1), i1 = (int)(p - (int64_t)i2 * n1);
    // offsets d with (d2 mod n2, d1 mod n1) == (i2, i1), d in [-R, R]^2 (several when the image is small)
    const int W = 2 * R + 1;
    T acc = T(0);
    for (int d2 = -R; d2 <= R; ++d2) {
        if (((d2 % n2) + n2) % n2 != i2) continue;
        for (int d1 = -R; d1 <= R; ++d1)
            if (((d1 % n1) + n1) % n1 == i1) acc += u[(int64_t)k * W * W + (d2 + R) * W + (d1 + R)];
    }
    out[e] = Cx<T>{acc, T(0)};
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_absmax(const Cx<T> *uh, int64_t N, T *mx)
{
    __shared__ T red[NTF];
    const Cx<T> *p = uh + (int64_t)blockIdx.x * N;
    T m = T(0);
    for (int64_t i = threadIdx.x; i < N; i += NTF) {
        const T a = sqrt(p[i].re * p[i].re + p[i].im * p[i].im);
        m = a > m ? a : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = NTF / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x + s] > red[threadIdx.x] ? red[threadIdx.x + s] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) mx[blockIdx.x] = red[0];
}

// gamma_k = mx_k / sum_j mx_j (1/m when every kernel is zero)
template <typename T>
__global__ void k_admm_gamma(const T *mx, int m, T *gam)
{
    const int k = threadIdx.x;
    if (k >= m) return;
    double tot = 0.0;
    for (int j = 0; j < m; ++j) tot += (double)mx[j];
    gam[k] = tot > 0.0 ? (T)((double)mx[k] / tot) : T(1) / (T)m;
}

// tw[t] = exp(-2 pi i t / n), t < n/2, evaluated in double
template <typename T>
__global__ void k_admm_twiddle(Cx<T> *tw, int n)
{
    const int t = blockIdx.x * NTF + threadIdx.x;
    if (t >= n / 2) return;
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)n, &sn, &cs);
    tw[t] = Cx<T>{(T)cs, (T)sn};
}

template <typename T>
__global__ void k_admm_diag(AdmmArgs<T> a)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    T mh = T(1), den = a.beta2;
    for (int k = 0; k < a.m; ++k) {
        const int64_t o = (int64_t)k * a.N + i;
        const Cx<T> u = a.uh[o];
        mh += (u.re * u.re + u.im * u.im) / (a.beta1 * a.gam[k]);
        den += a.beta1 * a.gam[k] * a.v[o] * a.v[o];
    }
    const_cast<T *>(a.mh)[i] = mh;
    const_cast<T *>(a.den)[i] = den;
}

template <typename T>
__global__ void k_admm_conjmul(const Cx<T> *uh_k, const Cx<T> *fh, Cx<T> *out, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= N) return;
    Cx<T> u = uh_k[i];
    u.im = -u.im;
    out[i] = cmul(u, fh[i]);
}

template <typename T>
__global__ void k_admm_real(const T *x, Cx<T> *out, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i < N) out[i] = Cx<T>{x[i], T(0)};
}

template <typename T>
__global__ void k_admm_takere(const Cx<T> *x, T *out, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i < N) out[i] = x[i].re;
}

}  // namespace

template <typename T>
hipError_t launch_fft2(Cx<T> *data, int n1, int n2, int batch, const Cx<T> *tw1, const Cx<T> *tw2, int inverse,
                       hipStream_t s)
{
    const int l1 = ilog2(n1), l2 = ilog2(n2);
    hipLaunchKernelGGL(k_fft_rows<T>, dim3(n2 * batch), dim3(NTF), 2 * n1 * sizeof(Cx<T>), s, data, n1, l1, tw1,
                       inverse);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // columns per workgroup: both LDS buffers within 64 KiB
    int cb = (int)(65536 / (2 * n2 * sizeof(Cx<T>)));
    cb = cb < 1 ? 1 : (cb > n1 ? n1 : cb);
    while (n1 % cb) --cb;
    const T scale = inverse ? T(1) / ((T)n1 * (T)n2) : T(1);
    hipLaunchKernelGGL(k_fft_cols<T>, dim3(n1 / cb, batch), dim3(NTF), 2 * cb * n2 * sizeof(Cx<T>), s, data, n1, n2,
                       l2, cb, tw2, inverse, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_admm_a(const AdmmArgs<T> &a, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_a<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a, k);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_acc(const AdmmArgs<T> &a, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_acc<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a, k);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_q(const AdmmArgs<T> &a, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_q<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a, k);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_g(const AdmmArgs<T> &a, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_g<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a, k);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_z(const AdmmArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_z<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_f(const AdmmArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_f<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_zeta(const AdmmArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_zeta<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_padk(const T *u, int R, int m, int n1, int n2, Cx<T> *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_padk<T>, dim3(nblk((int64_t)m * n1 * n2)), dim3(NTF), 0, s, u, R, m, n1, n2, out);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_absmax(const Cx<T> *uh, int m, int64_t N, T *mx, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_absmax<T>, dim3(m), dim3(NTF), 0, s, uh, N, mx);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_gamma(const T *mx, int m, T *gam, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_gamma<T>, dim3(1), dim3(64), 0, s, mx, m, gam);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_twiddle(Cx<T> *tw, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_twiddle<T>, dim3(nblk(n / 2)), dim3(NTF), 0, s, tw, n);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_diag(const AdmmArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_diag<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_conjmul(const Cx<T> *uh_k, const Cx<T> *fh, Cx<T> *out, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_conjmul<T>, dim3(nblk(N)), dim3(NTF), 0, s, uh_k, fh, out, N);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_real(const T *x, Cx<T> *out, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_real<T>, dim3(nblk(N)), dim3(NTF), 0, s, x, out, N);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_takere(const Cx<T> *x, T *out, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_takere<T>, dim3(nblk(N)), dim3(NTF), 0, s, x, out, N);
    return hipGetLastError();
}

#define PD_ADMM_INST(T)                                                                                       \
    template hipError_t launch_fft2<T>(Cx<T> *, int, int, int, const Cx<T> *, const Cx<T> *, int, hipStream_t); \
    template hipError_t launch_admm_a<T>(const AdmmArgs<T> &, int, hipStream_t);                              \
    template hipError_t launch_admm_acc<T>(const AdmmArgs<T> &, int, hipStream_t);                            \
    template hipError_t launch_admm_q<T>(const AdmmArgs<T> &, int, hipStream_t);                              \
    template hipError_t launch_admm_g<T>(const AdmmArgs<T> &, int, hipStream_t);                              \
    template hipError_t launch_admm_z<T>(const AdmmArgs<T> &, hipStream_t);                                   \
    template hipError_t launch_admm_f<T>(const AdmmArgs<T> &, hipStream_t);                                   \
    template hipError_t launch_admm_zeta<T>(const AdmmArgs<T> &, hipStream_t);                                \
    template hipError_t launch_admm_padk<T>(const T *, int, int, int, int, Cx<T> *, hipStream_t);             \
    template hipError_t launch_admm_absmax<T>(const Cx<T> *, int, int64_t, T *, hipStream_t);                 \
    template hipError_t launch_admm_gamma<T>(const T *, int, T *, hipStream_t);                               \
    template hipError_t launch_admm_twiddle<T>(Cx<T> *, int, hipStream_t);                                    \
    template hipError_t launch_admm_diag<T>(const AdmmArgs<T> &, hipStream_t);                                \
    template hipError_t launch_admm_conjmul<T>(const Cx<T> *, const Cx<T> *, Cx<T> *, int64_t, hipStream_t);  \
    template hipError_t launch_admm_real<T>(const T *, Cx<T> *, int64_t, hipStream_t);                        \
    template hipError_t launch_admm_takere<T>(const Cx<T> *, T *, int64_t, hipStream_t);
PD_ADMM_INST(float)
PD_ADMM_INST(double)

}  // namespace pd
