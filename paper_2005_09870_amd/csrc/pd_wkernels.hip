// pd_wkernels.hip -- gfx950 kernels of FISTA in the wavelet domain (FISTA-W /
// FISTA-WP, Section 4.3 and Appendix A.1).  One iteration is two products
// with the sparse matrix Theta_L (the paper's count of its cost):
//   u = Theta_L y(i) - z0                                  (k_wres)
//   g = Theta_L^T u, z(i) = Prox^Sigma(y(i) - tau Sigma g),
//   y(i+1) = z(i) + beta (z(i) - z(i-1))                   (k_wprox)
// The transpose is stored as its own CSR matrix so that both products gather
// (no atomics) and the prox and momentum fuse into the second product's row
// epilogue.  Both products are HBM-bound: the matrix streams once per
// product while the gathered vectors stay in L2 / the Infinity Cache.
//
// Row groups: G lanes (a power of two, picked from the average row length)
// share a row; lane j reads entries j, j+G, ... of it, UR per trip, and each
// group keeps NRG rows in flight together (their loads interleaved, all
// issued before the first use), so a wave has enough bytes outstanding to
// cover the three dependent latencies of a row (its bounds, its entries, the
// gathered values); the G partial sums meet in an xor tree.  A workgroup owns
// NRG x 256/G consecutive rows and writes their results through LDS as
// contiguous runs (whole cache lines, not one value per row group).
// Workgroups take consecutive row ranges in XCD-aware order, so each XCD's
// L2 sees a contiguous band of rows and the nearby columns they gather.
#include <hip/hip_runtime.h>

#include "pd_wkernels.h"

namespace pd {

namespace {

constexpr int NTW = 256;   // threads per workgroup (4 wave64)
constexpr int NXCDW = 8;

__device__ __forceinline__ int xcd_block(int total)
{
    const int b = blockIdx.x, per = (total + NXCDW - 1) / NXCDW;
    const int t = (b % NXCDW) * per + b / NXCDW;
    return t < total ? t : -1;
}
inline int xcd_blocks(int total) { return NXCDW * ((total + NXCDW - 1) / NXCDW); }

// Sum of NV doubles over the workgroup, added to slot (block % PD_NSLOT) of
// each of NV consecutive slot rows.
template <int NV>
__device__ void wblock_add(double (&v)[NV], double *slots)
{
    __shared__ double red[NV][NTW / 64];
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
        const int q = threadIdx.x;
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < NTW / 64; ++k) a += red[q][k];
        atomicAdd(slots + q * PD_NSLOT + (blockIdx.x % PD_NSLOT), a);
    }
}

// Row bounds clamped to [0, nnz] with b1 >= b0.
template <typename T>
__device__ __forceinline__ void row_bounds(const Csr<T> &A, int r, int64_t &b0, int64_t &b1)
{
    int64_t p = A.rp[r], q = A.rp[r + 1];
    p = p < 0 ? 0 : (p > A.nnz ? A.nnz : p);
    q = q < p ? p : (q > A.nnz ? A.nnz : q);
    b0 = p;
    b1 = q;
}

__device__ __forceinline__ int clamp_col(int c, int n) { return (unsigned)c < (unsigned)n ? c : (c < 0 ? 0 : n - 1); }

constexpr int UR = 4;    // entries per lane per trip
constexpr int NRG = 2;   // rows per lane group in flight together (4: fewer waves fit, slower)

// Partial sums of lane lg (0..G-1) over NRG rows [b0[j], b1[j]):
// sum val[k] x[col[k]]; the rows' loads are interleaved so that all of a
// trip's loads of every row are in flight before the first use.
template <typename T, int G>
__device__ __forceinline__ void rows_partial(const Csr<T> &A, const int64_t (&b0)[NRG], const int64_t (&b1)[NRG],
                                             const T *__restrict__ x, int lg, T (&acc)[NRG])
{
    int64_t k0[NRG];
#pragma unroll
    for (int j = 0; j < NRG; ++j) {
        acc[j] = T(0);
        k0[j] = b0[j];
    }
    for (;;) {
        bool more = false;
#pragma unroll
        for (int j = 0; j < NRG; ++j) more |= k0[j] < b1[j];
        if (!more) break;
        int ci[NRG][UR];
        T cv[NRG][UR];
        bool ok[NRG][UR];
#pragma unroll
        for (int j = 0; j < NRG; ++j)
#pragma unroll
            for (int q = 0; q < UR; ++q) {
                const int64_t k = k0[j] + q * G + lg;
                ok[j][q] = k < b1[j];
                const int64_t kk = ok[j][q] ? k : (b1[j] > b0[j] ? b1[j] - 1 : 0);  // in-range neighbour
                ci[j][q] = A.nnz > 0 ? A.col[kk] : 0;
                cv[j][q] = A.nnz > 0 ? A.val[kk] : T(0);
            }
        T xv[NRG][UR];
#pragma unroll
        for (int j = 0; j < NRG; ++j)
#pragma unroll
            for (int q = 0; q < UR; ++q) xv[j][q] = x[clamp_col(ci[j][q], A.n)];
#pragma unroll
        for (int j = 0; j < NRG; ++j) {
#pragma unroll
            for (int q = 0; q < UR; ++q) acc[j] = fma(ok[j][q] ? cv[j][q] : T(0), xv[j][q], acc[j]);
            k0[j] += UR * G;
        }
    }
}

// Sum over the G lanes of a group (aligned groups; every lane gets the sum).
template <typename T, int G>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// Band index k of Mallat position (i1, i2): 0 = coarsest approximation,
// 1..L detail bands from the coarsest level to the finest.
__device__ __forceinline__ int band_index(int i1, int i2, int n1, int n2, int L)
{
    int t1 = L, t2 = L;
    while (t1 > 0 && i1 >= (n1 >> t1)) --t1;
    while (t2 > 0 && i2 >= (n2 >> t2)) --t2;
    const int t = t1 < t2 ? t1 : t2;
    return t == L ? 0 : L - t;
}

template <typename T>
__device__ __forceinline__ T soft_w(T v, T t)
{
    T a = fabs(v) - t;
    return a > T(0) ? copysign(a, v) : T(0);
}

// Rows of lane group gi of workgroup blk: (blk * NRG + j) * RPB + gi, j < NRG
// (NRG RPB consecutive rows per workgroup).
template <typename T, int G>
__global__ __launch_bounds__(NTW) void k_wres(WResArgs<T> a)
{
    constexpr int RPB = NTW / G;
    __shared__ T su[NRG * RPB];
    const int nb = (a.a.n + RPB * NRG - 1) / (RPB * NRG);
    const int blk = xcd_block(nb);
    double st[1] = {0.0};
    if (blk >= 0) {
        const int lg = threadIdx.x & (G - 1), gi = threadIdx.x / G;
        int r[NRG];
        bool rok[NRG];
        T bv[NRG];
        int64_t b0[NRG], b1[NRG];
#pragma unroll
        for (int j = 0; j < NRG; ++j) {
            const int row = (blk * NRG + j) * RPB + gi;
            rok[j] = row < a.a.n;
            r[j] = rok[j] ? row : a.a.n - 1;
            bv[j] = a.b ? a.b[r[j]] : T(0);
            row_bounds(a.a, r[j], b0[j], b1[j]);
        }
        T acc[NRG];
        rows_partial<T, G>(a.a, b0, b1, a.x, lg, acc);
#pragma unroll
        for (int j = 0; j < NRG; ++j) {
            const T u = group_sum<T, G>(acc[j]) - bv[j];
            if (lg == 0) su[j * RPB + gi] = u;
            if (rok[j] && lg == 0) st[0] += 0.5 * (double)u * (double)u;
        }
        __syncthreads();
        const int row0 = blk * NRG * RPB;
        for (int t = threadIdx.x; t < NRG * RPB; t += NTW)
            if (row0 + t < a.a.n) a.u[row0 + t] = su[t];
    }
    if (a.slots) wblock_add<1>(st, a.slots);
}

template <typename T, int G>
__global__ __launch_bounds__(NTW) void k_wprox(WProxArgs<T> a)
{
    constexpr int RPB = NTW / G;
    __shared__ T sw[PD_MAXL + 1];
    __shared__ T sz[NRG * RPB], sy[NRG * RPB];
    const int nb = (a.at.n + RPB * NRG - 1) / (RPB * NRG);
    const int blk = xcd_block(nb);
    if (!a.wmap && threadIdx.x <= a.levels) sw[threadIdx.x] = a.wlev[threadIdx.x];
    double st[2] = {0.0, 0.0};
    bool bad = false;
    if (blk >= 0) {
        const int lg = threadIdx.x & (G - 1), gi = threadIdx.x / G;
        int r[NRG];
        bool rok[NRG];
        T y[NRG], zc[NRG], sg[NRG], wm[NRG];
        int64_t b0[NRG], b1[NRG];
#pragma unroll
        for (int j = 0; j < NRG; ++j) {  // the rows' own operands load while their entries stream
            const int row = (blk * NRG + j) * RPB + gi;
            rok[j] = row < a.at.n;
            r[j] = rok[j] ? row : a.at.n - 1;
            y[j] = a.y[r[j]];
            zc[j] = a.zc[r[j]];
            sg[j] = a.sigma ? a.sigma[r[j]] : T(1);
            wm[j] = a.wmap ? a.wmap[r[j]] : T(0);
            row_bounds(a.at, r[j], b0[j], b1[j]);
        }
        T acc[NRG];
        rows_partial<T, G>(a.at, b0, b1, a.u, lg, acc);
        __syncthreads();  // sw
#pragma unroll
        for (int j = 0; j < NRG; ++j) {
            const T g = group_sum<T, G>(acc[j]);
            T w = wm[j];
            if (!a.wmap) {
                const int i2 = r[j] / a.n1, i1 = r[j] - i2 * a.n1;
                w = sw[band_index(i1, i2, a.n1, a.n2, a.levels)];
            }
            const T ts = a.tau * sg[j];
            const T v = y[j] - ts * g;
            const T z = soft_w(v, ts * w);
            if (lg == 0) {
                sz[j * RPB + gi] = z;
                sy[j * RPB + gi] = fma(a.beta_next, z - zc[j], z);  // y(i+1), one explicit fma
            }
            if (rok[j] && lg == 0) {
                bad |= !isfinite(v);
                st[0] += (double)w * fabs((double)y[j]);
                st[1] += ((double)z - (double)y[j]) * ((double)z - (double)y[j]);
            }
        }
        __syncthreads();  // sz, sy
        const int row0 = blk * NRG * RPB;
        for (int t = threadIdx.x; t < NRG * RPB; t += NTW)
            if (row0 + t < a.at.n) {
                a.zn[row0 + t] = sz[t];
                a.y[row0 + t] = sy[t];
            }
    } else {
        __syncthreads();
    }
    if (a.slots) wblock_add<2>(st, a.slots + PD_NSLOT);
    if (bad) atomicOr(a.flag, 1);
}

template <typename T, int G>
__global__ __launch_bounds__(NTW) void k_wjacobi(Csr<T> at, T *sigma)
{
    constexpr int RPB = NTW / G;
    const int nb = (at.n + RPB - 1) / RPB;
    const int blk = xcd_block(nb);
    if (blk < 0) return;
    const int lg = threadIdx.x & (G - 1);
    const int row = blk * RPB + threadIdx.x / G;
    const bool rok = row < at.n;
    const int r = rok ? row : at.n - 1;
    int64_t b0, b1;
    row_bounds(at, r, b0, b1);
    T acc = T(0);
    for (int64_t k = b0 + lg; k < b1; k += G) {
        const T v = at.val[k];
        acc = fma(v, v, acc);
    }
    const T d = group_sum<T, G>(acc);
    if (rok && lg == 0) sigma[r] = d > T(0) ? T(1) / d : T(1);
}

template <typename T>
__global__ void k_wform_y(const T *zc, const T *zp, T beta, T *y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = fma(beta, zc[i] - zp[i], zc[i]);  // as the fused product
}

// ---------------------------------------------------------------- transpose --
__global__ void k_csr_check(const int64_t *rp, const int32_t *col, int n, int64_t nnz, int *flag)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t b0 = rp[r], b1 = rp[r + 1];
    bool bad = b0 < 0 || b1 < b0 || b1 > nnz || (r == 0 && b0 != 0) || (r == n - 1 && b1 != nnz);
    if (!bad) {
        int prev = -1;
        for (int64_t k = b0; k < b1; ++k) {
            const int c = col[k];
            if (c <= prev || c >= n) {
                bad = true;
                break;
            }
            prev = c;
        }
    }
    if (bad) atomicOr(flag, 1);
}

__global__ void k_fill_i32(int *p, int v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_csr_count(const int64_t *rp, const int32_t *col, int n, int *cnt)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (int64_t k = rp[r]; k < rp[r + 1]; ++k) atomicAdd(cnt + col[k], 1);
}

// Exclusive scan of cnt[0..n) into trp[0..n] by one workgroup: each thread
// sums a contiguous chunk, the chunk sums are scanned in LDS, then each
// thread writes its chunk's prefixes.
constexpr int NSCAN = 1024;
__global__ __launch_bounds__(NSCAN) void k_csr_scan(const int *cnt, int n, int64_t *trp)
{
    __shared__ int64_t part[NSCAN];
    const int t = threadIdx.x;
    const int per = (n + NSCAN - 1) / NSCAN;
    const int lo = t * per, hi = (lo + per < n) ? lo + per : n;
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < NSCAN; off <<= 1) {  // inclusive Hillis-Steele scan
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? part[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
        trp[i] = run;
        run += cnt[i];
    }
    if (t == NSCAN - 1) trp[n] = part[NSCAN - 1];
}

template <typename T>
__global__ void k_csr_scatter(Csr<T> a, const int64_t *trp, int *cur, int32_t *tcol, T *tval)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    for (int64_t k = a.rp[r]; k < a.rp[r + 1]; ++k) {
        const int c = a.col[k];
        const int64_t pos = trp[c] + atomicAdd(cur + c, 1);
        tcol[pos] = r;
        tval[pos] = a.val[k];
    }
}

// Insertion sort of each row of the transpose by column (the scatter order
// depends on atomic arrival; the sorted result does not).
template <typename T>
__global__ void k_csr_sort(const int64_t *trp, int n, int32_t *tcol, T *tval)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t b0 = trp[r], b1 = trp[r + 1];
    for (int64_t k = b0 + 1; k < b1; ++k) {
        const int c = tcol[k];
        const T v = tval[k];
        int64_t j = k - 1;
        while (j >= b0 && tcol[j] > c) {
            tcol[j + 1] = tcol[j];
            tval[j + 1] = tval[j];
            --j;
        }
        tcol[j + 1] = c;
        tval[j + 1] = v;
    }
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

int wgroup_for(int64_t nnz, int n)
{
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    if (avg <= 12.0) return 4;
    if (avg <= 24.0) return 8;
    if (avg <= 64.0) return 16;
    return 32;
}

#define PD_WDISPATCH(G, KER, ...)                                                           \
    switch (G) {                                                                            \
    case 4: hipLaunchKernelGGL((KER<T, 4>), __VA_ARGS__); break;                           \
    case 8: hipLaunchKernelGGL((KER<T, 8>), __VA_ARGS__); break;                           \
    case 16: hipLaunchKernelGGL((KER<T, 16>), __VA_ARGS__); break;                         \
    default: hipLaunchKernelGGL((KER<T, 32>), __VA_ARGS__); break;                         \
    }

template <typename T>
hipError_t launch_wres(const WResArgs<T> &a, int group, hipStream_t s)
{
    if (a.a.n <= 0) return hipSuccess;
    const int rows = (NTW / group) * NRG, nb = (a.a.n + rows - 1) / rows;
    PD_WDISPATCH(group, k_wres, dim3(xcd_blocks(nb)), dim3(NTW), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wprox(const WProxArgs<T> &a, int group, hipStream_t s)
{
    if (a.at.n <= 0) return hipSuccess;
    const int rows = (NTW / group) * NRG, nb = (a.at.n + rows - 1) / rows;
    PD_WDISPATCH(group, k_wprox, dim3(xcd_blocks(nb)), dim3(NTW), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wjacobi(const Csr<T> &at, T *sigma, int group, hipStream_t s)
{
    if (at.n <= 0) return hipSuccess;
    const int nb = (at.n + NTW / group - 1) / (NTW / group);
    PD_WDISPATCH(group, k_wjacobi, dim3(xcd_blocks(nb)), dim3(NTW), 0, s, at, sigma);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wform_y(const T *zc, const T *zp, T beta, T *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wform_y<T>, dim3(blocks_for(n, NTW)), dim3(NTW), 0, s, zc, zp, beta, y, n);
    return hipGetLastError();
}

hipError_t launch_csr_check(const int64_t *rp, const int32_t *col, int n, int64_t nnz, int *flag, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_check, dim3(blocks_for(n, NTW)), dim3(NTW), 0, s, rp, col, n, nnz, flag);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, NTW)), dim3(NTW), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_csr_count(const int64_t *rp, const int32_t *col, int n, int *cnt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_count, dim3(blocks_for(n, NTW)), dim3(NTW), 0, s, rp, col, n, cnt);
    return hipGetLastError();
}

hipError_t launch_csr_scan(const int *cnt, int n, int64_t *trp, hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_scan, dim3(1), dim3(NSCAN), 0, s, cnt, n, trp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_csr_scatter(const Csr<T> &a, const int64_t *trp, int *cur, int32_t *tcol, T *tval, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_scatter<T>, dim3(blocks_for(a.n, NTW)), dim3(NTW), 0, s, a, trp, cur, tcol, tval);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_csr_sort(const int64_t *trp, int n, int32_t *tcol, T *tval, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_csr_sort<T>, dim3(blocks_for(n, NTW)), dim3(NTW), 0, s, trp, n, tcol, tval);
    return hipGetLastError();
}

#define PD_WINST(T)                                                                                       \
    template hipError_t launch_wres<T>(const WResArgs<T> &, int, hipStream_t);                            \
    template hipError_t launch_wprox<T>(const WProxArgs<T> &, int, hipStream_t);                          \
    template hipError_t launch_wjacobi<T>(const Csr<T> &, T *, int, hipStream_t);                         \
    template hipError_t launch_wform_y<T>(const T *, const T *, T, T *, int64_t, hipStream_t);            \
    template hipError_t launch_csr_scatter<T>(const Csr<T> &, const int64_t *, int *, int32_t *, T *,     \
                                              hipStream_t);                                               \
    template hipError_t launch_csr_sort<T>(const int64_t *, int, int32_t *, T *, hipStream_t);
PD_WINST(float)
PD_WINST(double)

}  // namespace pd
