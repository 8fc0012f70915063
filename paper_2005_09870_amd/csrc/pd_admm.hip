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
// line FFT tiles: points per row tile, columns per column tile, threads per workgroup
constexpr int FFT_ROW_POINTS = 1024;
constexpr int FFT_COL_TILE = 4;
constexpr int FFT_THREADS = 256;
constexpr bool FFT_TW_LDS = true;  // twiddle table staged in LDS beside the tile

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

// ---- mixed-radix line FFT (lines of n >= 8 points) -------------------------
// Stockham autosort with one radix-2 or radix-4 stage first (when log2 n is not
// a multiple of 3) and radix-8 stages after it.  A thread owns "groups" of 8
// points: group g of a line holds positions g + t n/8 (t < 8), which are the
// inputs of one radix-8 butterfly, two radix-4 or four radix-2 ones.  The first
// stage reads the line from global memory and the last one writes it back
// (both at positions g + t n/8, so a line's loads and stores are contiguous);
// the stages in between exchange through one LDS tile, in place (all reads of
// a stage, barrier, all writes, barrier), padded by one point in every 8.  The inverse conjugates on load and
// store.

template <typename T>
__device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return Cx<T>{a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return Cx<T>{a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) { return Cx<T>{a.im, -a.re}; }  // a * (-i)

// X[q] = sum_r v[r] exp(-2 pi i r q / R), in place, natural order
template <typename T>
__device__ __forceinline__ void dft2(Cx<T> &a, Cx<T> &b)
{
    const Cx<T> t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename T>
__device__ __forceinline__ void dft4(Cx<T> &v0, Cx<T> &v1, Cx<T> &v2, Cx<T> &v3)
{
    const Cx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_mi(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft8(Cx<T> *v)
{
    Cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    Cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const T c = T(0.70710678118654752440);
    const Cx<T> w1{c * (o1.re + o1.im), c * (o1.im - o1.re)};    // o1 exp(-i pi/4)
    const Cx<T> w2 = mul_mi(o2);                                  // o2 exp(-i pi/2)
    const Cx<T> w3{c * (o3.im - o3.re), -c * (o3.re + o3.im)};   // o3 exp(-3 i pi/4)
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}

// exp(-2 pi i t / n) for t < n from the half table tw[t], t < n/2
template <typename T>
__device__ __forceinline__ Cx<T> twiddle(const Cx<T> *__restrict__ tw, int t, int half)
{
    if (t < half) return tw[t];
    const Cx<T> w = tw[t - half];
    return Cx<T>{-w.re, -w.im};
}

// One stage (radix R, Ns = product of the earlier radices) on the 8 points of
// group g: butterflies j = g + q n/8 (q < 8/R) with inputs v[q + r 8/R].
// Writes the outputs' positions into pos[] (same slots).
template <typename T, int R>
__device__ __forceinline__ void stage_group(Cx<T> *v, int *pos, int g, int n, int Ns,
                                            const Cx<T> *__restrict__ tw)
{
    constexpr int Q = 8 / R;
    const int n8 = n >> 3, stride = n / (Ns * R);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = g + q * n8;
        const int k = j & (Ns - 1);
        Cx<T> u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u[r] = v[q + r * Q];
            if (Ns > 1 && r > 0) u[r] = cmul(u[r], twiddle(tw, r * k * stride, n >> 1));
        }
        if constexpr (R == 8) {
            dft8(u);
        } else if constexpr (R == 4) {
            dft4(u[0], u[1], u[2], u[3]);
        } else {
            dft2(u[0], u[1]);
        }
        const int base = (j - k) * R + k;  // (j / Ns) Ns R + k
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[q + r * Q] = u[r];
            pos[q + r * Q] = base + r * Ns;
        }
    }
}

// C lines of n points per workgroup, BG groups per thread; grid (lines / C, batch).
// ROWS: line l is row (blockIdx.x C + l), points contiguous; else line l is
// column (blockIdx.x C + l), points n1 apart.  first: radix of the first stage.
template <typename T, bool ROWS, int BG>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_lines(Cx<T> *data, int n, int n1, int64_t plane, int C,
                                                  const Cx<T> *__restrict__ tw, int first, int nst,
                                                  int inverse, T scale)
{
    extern __shared__ unsigned char lds_raw[];
    Cx<T> *S = reinterpret_cast<Cx<T> *>(lds_raw);
    const int n8 = n >> 3, nthr = blockDim.x;
    Cx<T> *base = data + (int64_t)blockIdx.y * plane;
    // column tiles in XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so
    // workgroup b takes tile (b % 8) * per + b / 8 and the tiles that share cache lines (4
    // columns of 8 bytes each per 128-byte line) run on one XCD, from its L2
    int bx = blockIdx.x;
    if (!ROWS && (gridDim.x & 7) == 0) bx = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    const int line0 = bx * C;
    // tile index of point e of line l: one pad element every 8 points, so that the stride-8
    // writes of a radix-8 stage do not fall on the same banks
    const int np = n + (n >> 3);
    auto lidx = [&](int l, int e) { return ROWS ? l * np + e + (e >> 3) : (e + (e >> 3)) * C + l; };
    const Cx<T> *twp = tw;
    if (FFT_TW_LDS && nst > 1) {  // read first in stage 1, after its barrier
        Cx<T> *TW = S + C * np;
        for (int i = threadIdx.x; i < (n >> 1); i += nthr) TW[i] = tw[i];
        twp = TW;
    }
    Cx<T> v[BG][8];
    int pos[BG][8];
    int gl[BG], gg[BG];
    // load (positions g + t n/8)
#pragma unroll
    for (int b = 0; b < BG; ++b) {
        const int grp = threadIdx.x + b * nthr;
        gl[b] = ROWS ? grp / n8 : grp % C;
        gg[b] = ROWS ? grp % n8 : grp / C;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = gg[b] + t * n8;
            const int64_t off = ROWS ? (int64_t)(line0 + gl[b]) * n1 + e : (int64_t)e * n1 + line0 + gl[b];
            Cx<T> x = base[off];
            if (inverse) x.im = -x.im;
            v[b][t] = x;
        }
    }
    int Ns = 1;
    for (int s = 0; s < nst; ++s) {
        const int R = s == 0 ? first : 8;
        if (s > 0) {
            // gather this stage's inputs from the tile
            __syncthreads();
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int e = gg[b] + t * n8;
                    v[b][t] = S[lidx(gl[b], e)];
                }
            __syncthreads();
        }
#pragma unroll
        for (int b = 0; b < BG; ++b) {
            if (R == 8)
                stage_group<T, 8>(v[b], pos[b], gg[b], n, Ns, twp);
            else if (R == 4)
                stage_group<T, 4>(v[b], pos[b], gg[b], n, Ns, twp);
            else
                stage_group<T, 2>(v[b], pos[b], gg[b], n, Ns, twp);
        }
        Ns *= R;
        if (s + 1 < nst) {
#pragma unroll
            for (int b = 0; b < BG; ++b)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int e = pos[b][t];
                    S[lidx(gl[b], e)] = v[b][t];
                }
        }
    }
    // the last stage (radix 8) leaves point g + t n/8 in slot t: store
#pragma unroll
    for (int b = 0; b < BG; ++b)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int e = gg[b] + t * n8;
            const int64_t off = ROWS ? (int64_t)(line0 + gl[b]) * n1 + e : (int64_t)e * n1 + line0 + gl[b];
            Cx<T> x = v[b][t];
            if (inverse) x.im = -x.im;
            base[off] = Cx<T>{x.re * scale, x.im * scale};
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

// two partial sums to two slot rows (either may be nullptr) with one LDS round
__device__ void slots_add2(double v0, double *s0, double v1, double *s1)
{
    __shared__ double red[2][NTF / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        v0 += __shfl_xor(v0, m);
        v1 += __shfl_xor(v1, m);
    }
    if (lane == 0) {
        red[0][wv] = v0;
        red[1][wv] = v1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double *dst = threadIdx.x == 0 ? s0 : s1;
        if (dst) {
            double a = 0.0;
#pragma unroll
            for (int w = 0; w < NTF / 64; ++w) a += red[threadIdx.x][w];
            atomicAdd(dst + (blockIdx.x % PD_NSLOT), a);
        }
    }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + NTF - 1) / NTF); }

template <typename T>
__device__ __forceinline__ T pixel_weight(const AdmmArgs<T> &a, const T *sw, int64_t i)
{
    if (a.wmap) return a.wmap[i];
    const int i2 = (int)(i / a.n1), i1 = (int)(i - (int64_t)i2 * a.n1);
    return sw[band_of(i1, i2, a.n1, a.n2, a.levels)];
}

template <typename T>
__device__ __forceinline__ T soft_thr(T v, T t)
{
    const T m = fabs(v) - t;
    return m > T(0) ? copysign(m, v) : T(0);
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_a(AdmmArgs<T> a)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    const T f = a.f[i];
    for (int k = 0; k < a.m; ++k) {
        const int64_t o = (int64_t)k * a.N + i;
        const T ak = (a.utf0[o] - a.xi[o]) / (a.beta1 * a.gam[k]) + a.v[o] * f;
        a.g[o] = ak;
        a.cb[o] = Cx<T>{ak, T(0)};
    }
}

// M > 0: the term count as a compile-time constant (m <= 8), so that every term's operands are
// loaded before the first use; M == 0: any m, one term at a time.
template <typename T, int M>
__global__ __launch_bounds__(NTF) void k_admm_accq(AdmmArgs<T> a)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= a.N) return;
    Cx<T> t{T(0), T(0)};
    if constexpr (M > 0) {
        Cx<T> u[M], c[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            u[k] = a.uh[(int64_t)k * a.N + i];
            c[k] = a.cb[(int64_t)k * a.N + i];
        }
        const T im = T(1) / a.mh[i];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const Cx<T> p = cmul(u[k], c[k]);
            t.re += p.re;
            t.im += p.im;
        }
        t.re *= im;
        t.im *= im;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            Cx<T> w = u[k];
            w.im = -w.im;
            a.cb[(int64_t)k * a.N + i] = cmul(w, t);
        }
    } else {
        for (int k = 0; k < a.m; ++k) {
            const int64_t o = (int64_t)k * a.N + i;
            const Cx<T> p = cmul(a.uh[o], a.cb[o]);
            t.re += p.re;
            t.im += p.im;
        }
        const T im = T(1) / a.mh[i];
        t.re *= im;
        t.im *= im;
        for (int k = 0; k < a.m; ++k) {
            const int64_t o = (int64_t)k * a.N + i;
            Cx<T> u = a.uh[o];
            u.im = -u.im;
            a.cb[o] = cmul(u, t);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_z(AdmmArgs<T> a)
{
    __shared__ T sw[PD_MAXL + 1];
    if (!a.wmap && threadIdx.x <= a.levels) sw[threadIdx.x] = a.wlev[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    double st = 0.0;
    if (i < a.N) {
        const T w = pixel_weight(a, sw, i);
        const T zt = a.zeta[i];
        const T z = soft_thr(a.tz[i] - zt / a.beta2, w / a.beta2);
        a.z[i] = z;
        a.tf[i] = a.beta2 * z + zt;
        st = (double)w * fabs((double)z);
    }
    if (a.slots) slots_add2(st, a.slots + 2 * PD_NSLOT, 0.0, nullptr);
}

template <typename T, int M>
__global__ __launch_bounds__(NTF) void k_admm_f(AdmmArgs<T> a, int next)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    double st = 0.0;
    if (i < a.N) {
        if constexpr (M > 0) {
            T ak[M], cr[M], xk[M], vk[M], uf[M];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t o = (int64_t)k * a.N + i;
                ak[k] = a.g[o];
                cr[k] = a.cb[o].re;
                xk[k] = a.xi[o];
                vk[k] = a.v[o];
                uf[k] = a.utf0[o];
            }
            // g-step completion and f-step
            T gk[M];
            T acc = a.tfs[i];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const T bg = a.beta1 * a.gam[k];
                gk[k] = ak[k] - cr[k] / bg;
                acc += vk[k] * (xk[k] + bg * gk[k]);
            }
            const T f = acc / a.den[i];
            a.f[i] = f;
            // multiplier step, then the next iteration's a_k
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int64_t o = (int64_t)k * a.N + i;
                const T bg = a.beta1 * a.gam[k];
                const T r = gk[k] - vk[k] * f;
                const T x = xk[k] + bg * r;
                a.xi[o] = x;
                st += (double)a.gam[k] * (double)r * (double)r;
                if (next) {
                    const T an = (uf[k] - x) / bg + vk[k] * f;
                    a.g[o] = an;
                    a.cb[o] = Cx<T>{an, T(0)};
                }
            }
        } else {
            // g-step completion and f-step
            T acc = a.tfs[i];
            for (int k = 0; k < a.m; ++k) {
                const int64_t o = (int64_t)k * a.N + i;
                const T bg = a.beta1 * a.gam[k];
                const T gk = a.g[o] - a.cb[o].re / bg;
                acc += a.v[o] * (a.xi[o] + bg * gk);
            }
            const T f = acc / a.den[i];
            a.f[i] = f;
            // multiplier step, then the next iteration's a_k
            for (int k = 0; k < a.m; ++k) {
                const int64_t o = (int64_t)k * a.N + i;
                const T bg = a.beta1 * a.gam[k];
                const T vk = a.v[o];
                const T r = a.g[o] - a.cb[o].re / bg - vk * f;
                const T xk = a.xi[o] + bg * r;
                a.xi[o] = xk;
                st += (double)a.gam[k] * (double)r * (double)r;
                if (next) {
                    const T ak = (a.utf0[o] - xk) / bg + vk * f;
                    a.g[o] = ak;
                    a.cb[o] = Cx<T>{ak, T(0)};
                }
            }
        }
    }
    if (a.slots) slots_add2(st, a.slots, 0.0, nullptr);
}

template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_zeta(AdmmArgs<T> a, int next)
{
    __shared__ T sw[PD_MAXL + 1];
    if (next && !a.wmap && threadIdx.x <= a.levels) sw[threadIdx.x] = a.wlev[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    double st = 0.0, st2 = 0.0;
    if (i < a.N) {
        const T tz = a.tz[i];
        const T r = a.z[i] - tz;
        const T zt = a.zeta[i] + a.beta2 * r;
        a.zeta[i] = zt;
        st = (double)r * (double)r;
        if (next) {
            const T w = pixel_weight(a, sw, i);
            const T z = soft_thr(tz - zt / a.beta2, w / a.beta2);
            a.z[i] = z;
            a.tf[i] = a.beta2 * z + zt;
            st2 = (double)w * fabs((double)z);
        }
    }
    if (a.slots)
        slots_add2(st, a.slots + PD_NSLOT, st2, (next && a.slots_next) ? a.slots_next + 2 * PD_NSLOT : nullptr);
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

// mx[k] = max |u_k^| over the plane: grid (blocks, m), one atomic max per workgroup on the
// value's bit pattern (non-negative IEEE values order like their bits); mx zeroed first
template <typename T>
__global__ __launch_bounds__(NTF) void k_admm_absmax(const Cx<T> *uh, int64_t N, T *mx)
{
    __shared__ T red[NTF];
    const Cx<T> *p = uh + (int64_t)blockIdx.y * N;
    T m = T(0);
    for (int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x; i < N; i += (int64_t)gridDim.x * NTF) {
        const T a = sqrt(p[i].re * p[i].re + p[i].im * p[i].im);
        m = a > m ? a : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = NTF / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x + s] > red[threadIdx.x] ? red[threadIdx.x + s] : red[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if constexpr (sizeof(T) == 8)
            atomicMax(reinterpret_cast<unsigned long long *>(mx) + blockIdx.y, __double_as_longlong(red[0]));
        else
            atomicMax(reinterpret_cast<unsigned int *>(mx) + blockIdx.y, __float_as_uint(red[0]));
    }
}

template <typename T>
__global__ void k_fill_zero(T *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = T(0);
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
__global__ void k_admm_conjmul(const Cx<T> *uh, const Cx<T> *fh, Cx<T> *out, int m, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * NTF + threadIdx.x;
    if (i >= N) return;
    const Cx<T> x = fh[i];
    for (int k = 0; k < m; ++k) {
        Cx<T> u = uh[(int64_t)k * N + i];
        u.im = -u.im;
        out[(int64_t)k * N + i] = cmul(u, x);
    }
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

template <typename T, bool ROWS>
hipError_t launch_lines(Cx<T> *data, int n, int n1, int64_t plane, int lines, int C, int batch, const Cx<T> *tw,
                        int inverse, T scale, hipStream_t s)
{
    const int l = ilog2(n), rem = l % 3;
    const int first = rem == 1 ? 2 : (rem == 2 ? 4 : 8);
    const int nst = l / 3 + (rem ? 1 : 0);
    const int groups = C * (n >> 3);
    const int nthr = groups < FFT_THREADS ? groups : FFT_THREADS;
    const int bg = groups / nthr;
    // the kernel's indexing assumes C | lines, whole groups per thread and at most 4 of them
    if (C < 1 || lines % C || groups % nthr || (bg != 1 && bg != 2 && bg != 4)) return hipErrorInvalidValue;
    const size_t lds = nst > 1 ? ((size_t)C * (n + n / 8) + (FFT_TW_LDS ? n / 2 : 0)) * sizeof(Cx<T>) : 0;
    const dim3 grid(lines / C, batch);
    if (bg == 1)
        hipLaunchKernelGGL((k_fft_lines<T, ROWS, 1>), grid, dim3(nthr), lds, s, data, n, n1, plane, C, tw, first, nst,
                           inverse, scale);
    else if (bg == 2)
        hipLaunchKernelGGL((k_fft_lines<T, ROWS, 2>), grid, dim3(nthr), lds, s, data, n, n1, plane, C, tw, first, nst,
                           inverse, scale);
    else
        hipLaunchKernelGGL((k_fft_lines<T, ROWS, 4>), grid, dim3(nthr), lds, s, data, n, n1, plane, C, tw, first, nst,
                           inverse, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_pass(Cx<T> *data, int n1, int n2, int batch, const Cx<T> *tw, int inverse, int cols,
                           hipStream_t s)
{
    const T scale = (cols && inverse) ? T(1) / ((T)n1 * (T)n2) : T(1);
    const int64_t plane = (int64_t)n1 * n2;
    const int n = cols ? n2 : n1;
    const int lines = cols ? n1 : n2;
    if (n >= 8) {
        // tiles within 64 KiB of LDS and at most 4 groups of 8 points per thread; columns: at
        // most FFT_COL_TILE per tile so that a wide image still gives many workgroups
        const int cap = (int)(65536 / sizeof(Cx<T>)) - (FFT_TW_LDS ? n / 2 : 0);  // padded tile points
        int C = (cols ? 32 * FFT_THREADS : FFT_ROW_POINTS) / n;
        if (C * (n + n / 8) > cap) C = cap / (n + n / 8);
        if (C * n > 32 * FFT_THREADS) C = 32 * FFT_THREADS / n;
        if (cols && C > FFT_COL_TILE) C = FFT_COL_TILE;
        if (C > lines) C = lines;
        if (C < 1) C = 1;
        while (C & (C - 1)) C &= C - 1;  // a power of two (the LDS cap need not be one)
        if (cols) return launch_lines<T, false>(data, n, n1, plane, lines, C, batch, tw, inverse, scale, s);
        return launch_lines<T, true>(data, n, n1, plane, lines, C, batch, tw, inverse, scale, s);
    }
    if (!cols) {
        hipLaunchKernelGGL(k_fft_rows<T>, dim3(n2 * batch), dim3(NTF), 2 * n1 * sizeof(Cx<T>), s, data, n1,
                           ilog2(n1), tw, inverse);
        return hipGetLastError();
    }
    // short columns: cb columns per workgroup, both LDS buffers within 64 KiB
    int cb = (int)(65536 / (2 * n2 * sizeof(Cx<T>)));
    cb = cb < 1 ? 1 : (cb > n1 ? n1 : cb);
    while (n1 % cb) --cb;
    hipLaunchKernelGGL(k_fft_cols<T>, dim3(n1 / cb, batch), dim3(NTF), 2 * cb * n2 * sizeof(Cx<T>), s, data, n1,
                       n2, ilog2(n2), cb, tw, inverse, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft2(Cx<T> *data, int n1, int n2, int batch, const Cx<T> *tw1, const Cx<T> *tw2, int inverse,
                       hipStream_t s)
{
    hipError_t e = launch_fft_pass<T>(data, n1, n2, batch, tw1, inverse, 0, s);
    if (e != hipSuccess) return e;
    return launch_fft_pass<T>(data, n1, n2, batch, tw2, inverse, 1, s);
}

template <typename T>
hipError_t launch_admm_a(const AdmmArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_a<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_accq(const AdmmArgs<T> &a, hipStream_t s)
{
    const dim3 g(nblk(a.N)), b(NTF);
    switch (a.m) {
    case 1: hipLaunchKernelGGL((k_admm_accq<T, 1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_admm_accq<T, 2>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_admm_accq<T, 3>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_admm_accq<T, 4>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_admm_accq<T, 5>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_admm_accq<T, 6>), g, b, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_admm_accq<T, 7>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_admm_accq<T, 8>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_admm_accq<T, 0>), g, b, 0, s, a); break;
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_z(const AdmmArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_z<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_f(const AdmmArgs<T> &a, int next, hipStream_t s)
{
    const dim3 g(nblk(a.N)), b(NTF);
    switch (a.m) {
    case 1: hipLaunchKernelGGL((k_admm_f<T, 1>), g, b, 0, s, a, next); break;
    case 2: hipLaunchKernelGGL((k_admm_f<T, 2>), g, b, 0, s, a, next); break;
    case 3: hipLaunchKernelGGL((k_admm_f<T, 3>), g, b, 0, s, a, next); break;
    case 4: hipLaunchKernelGGL((k_admm_f<T, 4>), g, b, 0, s, a, next); break;
    case 5: hipLaunchKernelGGL((k_admm_f<T, 5>), g, b, 0, s, a, next); break;
    case 6: hipLaunchKernelGGL((k_admm_f<T, 6>), g, b, 0, s, a, next); break;
    case 7: hipLaunchKernelGGL((k_admm_f<T, 7>), g, b, 0, s, a, next); break;
    case 8: hipLaunchKernelGGL((k_admm_f<T, 8>), g, b, 0, s, a, next); break;
    default: hipLaunchKernelGGL((k_admm_f<T, 0>), g, b, 0, s, a, next); break;
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_admm_zeta(const AdmmArgs<T> &a, int next, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_zeta<T>, dim3(nblk(a.N)), dim3(NTF), 0, s, a, next);
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
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(1), dim3(64), 0, s, mx, m);
    int64_t nb = (N + NTF * 8 - 1) / (NTF * 8);
    if (nb > 256) nb = 256;
    hipLaunchKernelGGL(k_admm_absmax<T>, dim3((unsigned)nb, m), dim3(NTF), 0, s, uh, N, mx);
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
hipError_t launch_admm_conjmul(const Cx<T> *uh, const Cx<T> *fh, Cx<T> *out, int m, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_admm_conjmul<T>, dim3(nblk(N)), dim3(NTF), 0, s, uh, fh, out, m, N);
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
    template hipError_t launch_fft_pass<T>(Cx<T> *, int, int, int, const Cx<T> *, int, int, hipStream_t);     \
    template hipError_t launch_admm_a<T>(const AdmmArgs<T> &, hipStream_t);                                   \
    template hipError_t launch_admm_accq<T>(const AdmmArgs<T> &, hipStream_t);                                \
    template hipError_t launch_admm_z<T>(const AdmmArgs<T> &, hipStream_t);                                   \
    template hipError_t launch_admm_f<T>(const AdmmArgs<T> &, int, hipStream_t);                              \
    template hipError_t launch_admm_zeta<T>(const AdmmArgs<T> &, int, hipStream_t);                           \
    template hipError_t launch_admm_padk<T>(const T *, int, int, int, int, Cx<T> *, hipStream_t);             \
    template hipError_t launch_admm_absmax<T>(const Cx<T> *, int, int64_t, T *, hipStream_t);                 \
    template hipError_t launch_admm_gamma<T>(const T *, int, T *, hipStream_t);                               \
    template hipError_t launch_admm_twiddle<T>(Cx<T> *, int, hipStream_t);                                    \
    template hipError_t launch_admm_diag<T>(const AdmmArgs<T> &, hipStream_t);                                \
    template hipError_t launch_admm_conjmul<T>(const Cx<T> *, const Cx<T> *, Cx<T> *, int, int64_t, hipStream_t); \
    template hipError_t launch_admm_real<T>(const T *, Cx<T> *, int64_t, hipStream_t);                        \
    template hipError_t launch_admm_takere<T>(const Cx<T> *, T *, int64_t, hipStream_t);
PD_ADMM_INST(float)
PD_ADMM_INST(double)

}  // namespace pd
