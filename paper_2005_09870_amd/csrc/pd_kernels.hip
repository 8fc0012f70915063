// pd_kernels.hip -- gfx950 kernels of the FISTA-Spa iteration for the
// wavelet-l1 deblurring energy (Escande & Weiss, arXiv:2005.09870, eq. 4.1,
// Appendix A.1).  One iteration is
//
//   synthesis  x = Psi y            (inverse periodic 2-D FWT, coarse -> fine)
//   blur       s = H^T (H x - f0)   (row-separable spatially varying blur)
//   analysis   g = Psi^* s          (forward FWT, fine -> coarse), with the
//              gradient step, soft threshold and momentum fused into the
//              writes of every band.
//
// Every kernel works on one LDS tile per workgroup (256 threads = 4 wave64),
// loads its halo with periodic wrap, and accumulates FP64 statistics with one
// atomic per workgroup.  Filters are zero-padded to 12 taps so any even
// length <= 12 runs the same code.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pd_kernels.h"

namespace pd {

constexpr int NT = 256;  // threads per workgroup

__device__ __forceinline__ int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Block-wide sum of up to three doubles, added atomically to dst[0..n-1].
template <int NV>
__device__ void block_atomic_add(double (&v)[NV], double *dst)
{
    __shared__ double red[NV][NT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double a = v[q];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) red[q][wv] = a;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double a = 0.0;
        for (int k = 0; k < NT / 64; ++k) a += red[threadIdx.x][k];
        atomicAdd(dst + threadIdx.x, a);
    }
}

// Soft threshold S_t(v) = sign(v) max(|v| - t, 0), zero on |v| <= t.
template <typename T>
__device__ __forceinline__ T soft(T v, T t)
{
    T a = fabs(v) - t;
    return a > T(0) ? copysign(a, v) : T(0);
}

// ---------------------------------------------------------------------------
// Synthesis of one level (Section 2.1 expansion, separable along x2 then x1):
//   fine[n] = sum_l h[n-2l] lo[l] + g[n-2l] hi[l],
// for output n = 2p + par the low-pass terms are l = p-5+j with tap
// h[par+10-2j] and the high-pass terms l = p+j with tap g[par-2j], j = 0..5.
// A workgroup produces a (2*TP2) x (2*TP1) tile of the finer approximation.
// ---------------------------------------------------------------------------
constexpr int SP1 = 32, SP2 = 16;               // coarse tile per band
constexpr int SR1 = SP1 + 10, SR2 = SP2 + 10;   // with halo
constexpr int SF1 = 2 * SP1, SF2 = 2 * SP2;     // fine tile

template <typename T>
__global__ __launch_bounds__(NT) void k_synth(SynthArgs<T> a)
{
    __shared__ T sB[4][SR2][SR1 + 1];  // LL, HL (hi x1), LH (hi x2), HH
    __shared__ T sLH[2][SF2][SR1 + 1]; // after x2 synthesis: low / high along x1
    const int M1c = a.M1c, M2c = a.M2c;
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int64_t ch = blockIdx.z;
    const int p01 = blockIdx.x * SP1, p02 = blockIdx.y * SP2;

    const T *zc = a.zc + ch * a.plane;
    const T *zp = a.zp + ch * a.plane;
    const T *apx = a.apx ? a.apx + ch * a.apx_plane : nullptr;
    const T beta = a.beta;

    for (int e = threadIdx.x; e < 4 * SR2 * SR1; e += NT) {
        int b = e / (SR2 * SR1), rem = e - b * SR2 * SR1;
        int r = rem / SR1, c = rem - r * SR1;
        int q2 = wrap(p02 - 5 + r, M2c), q1 = wrap(p01 - 5 + c, M1c);
        T v;
        if (b == 0 && apx) {
            v = apx[(int64_t)q2 * M1c + q1];
        } else {
            int row = q2 + ((b & 2) ? M2c : 0);
            int col = q1 + ((b & 1) ? M1c : 0);
            int64_t idx = (int64_t)row * a.pitch + col;
            T zcv = zc[idx];
            v = zcv + beta * (zcv - zp[idx]);
        }
        sB[b][r][c] = v;
    }
    __syncthreads();

    // along x2: low band (LL, LH) and high band (HL, HH), fine rows f
    for (int e = threadIdx.x; e < 2 * SF2 * SR1; e += NT) {
        int band = e / (SF2 * SR1), rem = e - band * SF2 * SR1;
        int f = rem / SR1, c = rem - f * SR1;
        int pl = f >> 1, par = f & 1;
        const int bl = band ? 1 : 0, bh = band ? 3 : 2;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            acc = fma(a.f.h[par + 10 - 2 * j], sB[bl][pl + j][c], acc);
            acc = fma(a.f.g[par - 2 * j + 10], sB[bh][pl + 5 + j][c], acc);
        }
        sLH[band][f][c] = acc;
    }
    __syncthreads();

    // along x1
    T *out = a.out + ch * a.out_plane;
    for (int e = threadIdx.x; e < SF2 * SF1; e += NT) {
        int f = e / SF1, c = e - f * SF1;
        int pl = c >> 1, par = c & 1;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            acc = fma(a.f.h[par + 10 - 2 * j], sLH[0][f][pl + j], acc);
            acc = fma(a.f.g[par - 2 * j + 10], sLH[1][f][pl + 5 + j], acc);
        }
        int o2 = 2 * p02 + f, o1 = 2 * p01 + c;
        if (o2 < M2 && o1 < M1) out[(int64_t)o2 * a.out_pitch + o1] = acc;
    }
}

// ---------------------------------------------------------------------------
// Analysis of one level (Section 2.1):
//   lo[l] = sum_{k=0}^{11} h[k] in[2l+k],  hi[l] = sum_{k=-10}^{1} g[k] in[2l+k]
// along x1 then x2.  A workgroup produces a TC2 x TC1 tile of each band; the
// detail bands (and, at the coarsest level, the approximation band) go
// through the fused gradient step + prox + momentum, or are stored plainly.
// ---------------------------------------------------------------------------
constexpr int TC1 = 32, TC2 = 16;
constexpr int AR1 = 2 * TC1 + 20, AR2 = 2 * TC2 + 20;  // fine region incl. halo

template <typename T>
__global__ __launch_bounds__(NT) void k_analysis(AnalysisArgs<T> a)
{
    __shared__ T sIn[AR2][AR1 + 1];
    __shared__ T sRow[2][AR2][TC1 + 1];   // low / high along x1
    __shared__ T sRes[PD_MAXC][4][TC2][TC1 + 1];
    const int M1c = a.M1c, M2c = a.M2c;
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int c01 = blockIdx.x * TC1, c02 = blockIdx.y * TC2;
    const int cbeg = a.joint ? 0 : blockIdx.z;
    const int cend = a.joint ? a.C : blockIdx.z + 1;

    for (int ch = cbeg; ch < cend; ++ch) {
        const T *in = a.in + (int64_t)ch * a.in_plane;
        for (int e = threadIdx.x; e < AR2 * AR1; e += NT) {
            int r = e / AR1, c = e - r * AR1;
            int q2 = wrap(2 * c02 - 10 + r, M2), q1 = wrap(2 * c01 - 10 + c, M1);
            sIn[r][c] = in[(int64_t)q2 * a.in_pitch + q1];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * AR2 * TC1; e += NT) {
            int band = e / (AR2 * TC1), rem = e - band * AR2 * TC1;
            int r = rem / TC1, l = rem - r * TC1;
            T acc = T(0);
            if (band == 0) {
#pragma unroll
                for (int k = 0; k < 12; ++k) acc = fma(a.f.h[k], sIn[r][2 * l + k + 10], acc);
            } else {
#pragma unroll
                for (int k = -10; k <= 1; ++k) acc = fma(a.f.g[k + 10], sIn[r][2 * l + k + 10], acc);
            }
            sRow[band][r][l] = acc;
        }
        __syncthreads();
        const int cc = a.joint ? ch : 0;
        for (int e = threadIdx.x; e < 4 * TC2 * TC1; e += NT) {
            int b = e / (TC2 * TC1), rem = e - b * TC2 * TC1;
            int l2 = rem / TC1, l1 = rem - l2 * TC1;
            const int src = b & 1;       // bit 0: high along x1
            const bool hi2 = (b & 2) != 0; // bit 1: high along x2
            T acc = T(0);
            if (!hi2) {
#pragma unroll
                for (int k = 0; k < 12; ++k) acc = fma(a.f.h[k], sRow[src][2 * l2 + k + 10][l1], acc);
            } else {
#pragma unroll
                for (int k = -10; k <= 1; ++k) acc = fma(a.f.g[k + 10], sRow[src][2 * l2 + k + 10][l1], acc);
            }
            sRes[cc][b][l2][l1] = acc;
        }
        __syncthreads();
    }

    // outputs
    double st[2] = {0.0, 0.0};  // sum w|y|, sum (z-y)^2
    bool bad = false;
    const bool last = a.last;
    for (int e = threadIdx.x; e < 4 * TC2 * TC1; e += NT) {
        int b = e / (TC2 * TC1), rem = e - b * TC2 * TC1;
        int l2 = rem / TC1, l1 = rem - l2 * TC1;
        int g2 = c02 + l2, g1 = c01 + l1;
        if (g2 >= M2c || g1 >= M1c) continue;
        if (b == 0 && !last) {  // intermediate approximation band
            for (int ch = cbeg; ch < cend; ++ch)
                a.apx_out[(int64_t)ch * a.apx_plane + (int64_t)g2 * M1c + g1] =
                    sRes[a.joint ? ch : 0][0][l2][l1];
            continue;
        }
        int row = g2 + ((b & 2) ? M2c : 0);
        int col = g1 + ((b & 1) ? M1c : 0);
        int64_t idx = (int64_t)row * a.pitch + col;
        if (a.mode == MODE_PLAIN) {
            for (int ch = cbeg; ch < cend; ++ch)
                a.zn[(int64_t)ch * a.plane + idx] = sRes[a.joint ? ch : 0][b][l2][l1];
            continue;
        }
        const int band = (b == 0) ? 0 : a.band_detail;  // band index k
        const T tau = a.tau;
        if (!a.joint) {
            const int64_t ci = (int64_t)blockIdx.z * a.plane + idx;
            T zcv = a.zc[ci];
            T y = zcv + a.beta * (zcv - a.zp[ci]);
            T w = a.wmap ? a.wmap[ci] : a.wlev[band];
            T v = y - tau * sRes[0][b][l2][l1];
            T z = soft(v, tau * w);
            a.zn[ci] = z;
            bad |= !isfinite(v);
            st[0] += (double)w * fabs((double)y);
            st[1] += ((double)z - (double)y) * ((double)z - (double)y);
        } else {
            T yv[PD_MAXC], vv[PD_MAXC];
            T nv = T(0);
            double ny = 0.0;
            for (int ch = 0; ch < a.C; ++ch) {
                const int64_t ci = (int64_t)ch * a.plane + idx;
                T zcv = a.zc[ci];
                yv[ch] = zcv + a.beta * (zcv - a.zp[ci]);
                vv[ch] = yv[ch] - tau * sRes[ch][b][l2][l1];
                nv = fma(vv[ch], vv[ch], nv);
                ny += (double)yv[ch] * (double)yv[ch];
            }
            T w = a.wlev[band];
            T nrm = sqrt(nv);
            T sc = nrm > T(0) ? T(1) - tau * w / nrm : T(0);
            sc = sc > T(0) ? sc : T(0);
            bad |= !isfinite(nrm);
            st[0] += (double)w * sqrt(ny);
            for (int ch = 0; ch < a.C; ++ch) {
                T z = vv[ch] * sc;
                a.zn[(int64_t)ch * a.plane + idx] = z;
                st[1] += ((double)z - (double)yv[ch]) * ((double)z - (double)yv[ch]);
            }
        }
    }
    if (a.mode == MODE_PROX) {
        if (a.stats) block_atomic_add<2>(st, a.stats + 1);
        if (bad) atomicOr(a.flag, 1);
    }
}

// ---------------------------------------------------------------------------
// Blur (Section 1, eq. 1.1; Operator 1 of Section 4.1): with the profile
// k_{y2} of source row y2,
//   t(x1,y2)  = sum_d k_{y2}[d] x(x1-d, y2)             (rows, own profile)
//   Hx(x1,x2) = sum_d k_{x2-d}[d] t(x1, x2-d)           (columns, source profile)
//   r = Hx - f0
//   u(x1,y2)  = sum_d k_{y2}[d] r(x1, y2+d)             (H^T: columns)
//   s(y1,y2)  = sum_d k_{y2}[d] u(y1+d, y2)             (H^T: rows)
// One workgroup produces a BT2 x BT1 tile of s; RM = 9 is the largest
// half-width (profiles narrower than that are zero-padded).
// ---------------------------------------------------------------------------
constexpr int RM = PD_MAX_RADIUS;
constexpr int BT1 = 64, BT2 = 32;
constexpr int BX1 = BT1 + 4 * RM, BX2 = BT2 + 4 * RM;  // x region
constexpr int BU1 = BT1 + 2 * RM;                       // t, r, u columns
constexpr int BR2 = BT2 + 2 * RM;                       // r rows

template <typename T>
__global__ __launch_bounds__(NT) void k_blur(BlurArgs<T> a)
{
    // sA: x (BX2 x BX1), later r (BR2 x BU1); sB: t (BX2 x BU1), later u (BT2 x BU1)
    __shared__ T sA[BX2 * BX1];
    __shared__ T sB[BX2 * BU1];
    __shared__ T sK[BX2][2 * RM + 1];
    const int n1 = a.n1, n2 = a.n2, R = a.R;
    const int64_t ch = blockIdx.z;
    const int o1 = blockIdx.x * BT1, o2 = blockIdx.y * BT2;
    const T *x = a.x + ch * a.plane;
    const T *f0 = a.f0 + ch * a.plane;

    for (int e = threadIdx.x; e < BX2 * (2 * RM + 1); e += NT) {
        int r = e / (2 * RM + 1), d = e - r * (2 * RM + 1) - RM;
        int row = wrap(o2 - 2 * RM + r, n2);
        sK[r][d + RM] = (d >= -R && d <= R) ? a.taps[(int64_t)row * (2 * R + 1) + d + R] : T(0);
    }
    for (int e = threadIdx.x; e < BX2 * BX1; e += NT) {
        int r = e / BX1, c = e - r * BX1;
        int q2 = wrap(o2 - 2 * RM + r, n2), q1 = wrap(o1 - 2 * RM + c, n1);
        sA[e] = x[(int64_t)q2 * n1 + q1];
    }
    __syncthreads();
    // t on rows [0,BX2) (pixel row o2-2RM+r), cols [0,BU1) (pixel col o1-RM+c)
    for (int e = threadIdx.x; e < BX2 * BU1; e += NT) {
        int r = e / BU1, c = e - r * BU1;
        T acc = T(0);
#pragma unroll
        for (int d = -RM; d <= RM; ++d) acc = fma(sK[r][d + RM], sA[r * BX1 + c + RM - d], acc);
        sB[e] = acc;
    }
    __syncthreads();
    // r on rows [0,BR2) (pixel row o2-RM+r), cols [0,BU1)
    double st[1] = {0.0};
    for (int e = threadIdx.x; e < BR2 * BU1; e += NT) {
        int r = e / BU1, c = e - r * BU1;
        T acc = T(0);
#pragma unroll
        for (int d = -RM; d <= RM; ++d)  // source row (x2 - d) has local index r + RM - d
            acc = fma(sK[r + RM - d][d + RM], sB[(r + RM - d) * BU1 + c], acc);
        int q2 = wrap(o2 - RM + r, n2), q1 = wrap(o1 - RM + c, n1);
        T rv = acc - f0[(int64_t)q2 * n1 + q1];
        sA[e] = rv;
        bool own = r >= RM && r < RM + BT2 && c >= RM && c < RM + BT1 &&
                   (o2 - RM + r) < n2 && (o1 - RM + c) < n1;
        if (own) st[0] += 0.5 * (double)rv * (double)rv;
    }
    __syncthreads();
    // u on rows [0,BT2) (pixel row o2+r), cols [0,BU1)
    for (int e = threadIdx.x; e < BT2 * BU1; e += NT) {
        int r = e / BU1, c = e - r * BU1;
        T acc = T(0);
#pragma unroll
        for (int d = -RM; d <= RM; ++d) acc = fma(sK[r + 2 * RM][d + RM], sA[(r + RM + d) * BU1 + c], acc);
        sB[e] = acc;
    }
    __syncthreads();
    T *s = a.s + ch * a.plane;
    for (int e = threadIdx.x; e < BT2 * BT1; e += NT) {
        int r = e / BT1, c = e - r * BT1;
        T acc = T(0);
#pragma unroll
        for (int d = -RM; d <= RM; ++d) acc = fma(sK[r + 2 * RM][d + RM], sB[r * BU1 + c + RM + d], acc);
        int q2 = o2 + r, q1 = o1 + c;
        if (q2 < n2 && q1 < n1) s[(int64_t)q2 * n1 + q1] = acc;
    }
    if (a.stats) block_atomic_add<1>(st, a.stats);
}

// H = Id: s = r = x - f0.
template <typename T>
__global__ __launch_bounds__(NT) void k_identity(BlurArgs<T> a)
{
    double st[1] = {0.0};
    const int64_t total = (int64_t)a.n1 * a.n2 * a.C;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
        T rv = a.x[e] - a.f0[e];
        a.s[e] = rv;
        st[0] += 0.5 * (double)rv * (double)rv;
    }
    if (a.stats) block_atomic_add<1>(st, a.stats);
}

// Single blur pass H or H^T (building block; not on the iteration path).
template <typename T>
__global__ __launch_bounds__(NT) void k_blur_single(BlurArgs<T> a, int transpose)
{
    const int64_t total = (int64_t)a.n1 * a.n2;
    const int64_t ch = blockIdx.y;
    const T *x = a.x + ch * a.plane;
    T *s = a.s + ch * a.plane;
    const int n1 = a.n1, n2 = a.n2, R = a.R, W = 2 * R + 1;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
        int i2 = (int)(e / n1), i1 = (int)(e - (int64_t)i2 * n1);
        T acc = T(0);
        if (!transpose) {
            for (int d2 = -R; d2 <= R; ++d2) {
                int y2 = wrap(i2 - d2, n2);
                const T *k = a.taps + (int64_t)y2 * W + R;
                T t = T(0);
                for (int d1 = -R; d1 <= R; ++d1) t = fma(k[d1], x[(int64_t)y2 * n1 + wrap(i1 - d1, n1)], t);
                acc = fma(k[d2], t, acc);
            }
        } else {
            const T *k = a.taps + (int64_t)i2 * W + R;
            for (int d2 = -R; d2 <= R; ++d2) {
                int x2 = wrap(i2 + d2, n2);
                T t = T(0);
                for (int d1 = -R; d1 <= R; ++d1) t = fma(k[d1], x[(int64_t)x2 * n1 + wrap(i1 + d1, n1)], t);
                acc = fma(k[d2], t, acc);
            }
        }
        s[e] = acc;
    }
}

template <typename T>
__global__ void k_copy(const T *src, T *dst, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

// ------------------------------------------------------------ launchers ---
template <typename T>
hipError_t launch_synth(const SynthArgs<T> &a, int C, hipStream_t s)
{
    dim3 grid((a.M1c + SP1 - 1) / SP1, (a.M2c + SP2 - 1) / SP2, C);
    hipLaunchKernelGGL(k_synth<T>, grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_analysis(const AnalysisArgs<T> &a, hipStream_t s)
{
    dim3 grid((a.M1c + TC1 - 1) / TC1, (a.M2c + TC2 - 1) / TC2, a.joint ? 1 : a.C);
    hipLaunchKernelGGL(k_analysis<T>, grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blur(const BlurArgs<T> &a, bool identity, hipStream_t s)
{
    if (identity) {
        int64_t total = (int64_t)a.n1 * a.n2 * a.C;
        int blocks = (int)((total + NT - 1) / NT);
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_identity<T>, dim3(blocks), dim3(NT), 0, s, a);
    } else {
        dim3 grid((a.n1 + BT1 - 1) / BT1, (a.n2 + BT2 - 1) / BT2, a.C);
        hipLaunchKernelGGL(k_blur<T>, grid, dim3(NT), 0, s, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blur_single(const BlurArgs<T> &a, int transpose, hipStream_t s)
{
    int64_t total = (int64_t)a.n1 * a.n2;
    int blocks = (int)((total + NT - 1) / NT);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_blur_single<T>, dim3(blocks, a.C), dim3(NT), 0, s, a, transpose);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy<T>, dim3(blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

#define PD_INST(T)                                                                          \
    template hipError_t launch_synth<T>(const SynthArgs<T> &, int, hipStream_t);           \
    template hipError_t launch_analysis<T>(const AnalysisArgs<T> &, hipStream_t);          \
    template hipError_t launch_blur<T>(const BlurArgs<T> &, bool, hipStream_t);            \
    template hipError_t launch_blur_single<T>(const BlurArgs<T> &, int, hipStream_t);      \
    template hipError_t launch_copy<T>(const T *, T *, int64_t, hipStream_t);
PD_INST(float)
PD_INST(double)

}  // namespace pd
