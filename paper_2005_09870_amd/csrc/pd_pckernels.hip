// pd_pckernels.hip -- gfx950 kernels of the product-convolution operator
//   H f = sum_k u_k * (v_k . f),   H^T r = sum_k v_k . (u_k (x) r)
// (Section 1's expansion, Section 3.1; FISTA-PC of Table 1), with
// (u * g)(p) = sum_d u(d) g(p - d) and (u (x) r)(p) = sum_d u(d) r(p + d),
// periodic, d in [-R, R]^2.
//
// k_pcblur fuses r = H x - f0 and s = H^T r on a 32 x 32 output tile: the x
// region (tile + 2R each side, staged in LDS once) is multiplied by one
// multiplier at a time and convolved into the r region (tile + R each side,
// accumulated in registers); then r (in LDS) is correlated with each kernel
// and weighted by the multiplier at the output.  Both sweeps are direct 2-D
// stencils of (2R+1)^2 taps per term, register-blocked along columns: a
// thread owns a column segment of the region (10 rows of r, 4 of s) and reads
// one window of that column per kernel column, so each LDS value feeds up to
// 2R+1 FMAs.  Taps are padded to R = 9 with zeros.  ALU-bound: 2 x m x 361
// FMA per pixel, plus the r halo (50^2 / 32^2 = 2.44x on the first sweep).
#include <hip/hip_runtime.h>

#include "pd_pckernels.h"

namespace pd {

namespace {

constexpr int PR = PD_MAX_RADIUS;   // 9: taps padded to (2PR+1)^2
constexpr int PW = 2 * PR + 1;      // 19
constexpr int PT = 32;              // output tile (both axes)
constexpr int RG = PT + 2 * PR;     // 50: r region
constexpr int XG = PT + 4 * PR;     // 68: x region
constexpr int PXP = XG + 1;         // LDS pitches
constexpr int PRP = RG + 1;
// Thread layouts (NTP threads; a thread owns RSEG rows of one r column and SSEG rows of one s column):
// 256 threads (10 / 4 rows) when the image has many tiles, 512 (5 / 2) when few tiles must fill the chip.
template <int NTP, int RSEG, int SSEG>
struct PcLayout {
    static constexpr int nt = NTP, rseg = RSEG, sseg = SSEG;
    static constexpr int XPT = (XG * XG + NTP - 1) / NTP;  // x-region elements per thread
    static_assert(RG % RSEG == 0 && RG * (RG / RSEG) <= NTP && PT * (PT / SSEG) == NTP, "pc tile tasks");
};
using PcSmall = PcLayout<256, 10, 4>;
using PcLarge = PcLayout<512, 5, 2>;

__device__ __forceinline__ int wrapp(int a, int n)
{
    if (a >= 0 && a < n) return a;
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Taps of term k padded to PR (zero outside radius R) into sU.
template <typename T, int NTP>
__device__ __forceinline__ void load_taps(const PcArgs<T> &a, int k, T *sU)
{
    const int W = 2 * a.R + 1;
    for (int e = threadIdx.x; e < PW * PW; e += NTP) {
        const int p = e / PW, q = e - p * PW;  // (d2, d1) + PR
        const int d2 = p - PR, d1 = q - PR;
        const bool in = d2 >= -a.R && d2 <= a.R && d1 >= -a.R && d1 <= a.R;
        sU[e] = in ? a.u[(int64_t)k * W * W + (d2 + a.R) * W + (d1 + a.R)] : T(0);
    }
}

template <typename T, int NTP>
__device__ void block_add1(double v, double *slots)
{
    __shared__ double red[NTP / 64];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NTP / 64; ++w) t += red[w];
        const unsigned blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        atomicAdd(slots + (blk % PD_NSLOT), t);
    }
}

template <typename T, class LY>
__global__ __launch_bounds__(LY::nt) void k_pcblur(PcArgs<T> a)
{
    constexpr int NTP = LY::nt, RSEG = LY::rseg, SSEG = LY::sseg, XPT = LY::XPT;
    __shared__ T sX[XG][PXP];
    __shared__ T sG[XG][PXP];
    __shared__ T sU[PW * PW];
    __shared__ T sR[RG][PRP];
    const int n1 = a.n1, n2 = a.n2;
    const int o1 = blockIdx.x * PT, o2 = blockIdx.y * PT;
    const int64_t ch = blockIdx.z;
    const T *x = a.x + ch * a.plane;
    const int tid = threadIdx.x;

    // x region: pixel (o2 - 2PR + i, o1 - 2PR + j), periodic
    for (int e = tid; e < XG * XG; e += NTP) {
        const int i = e / XG, j = e - i * XG;
        sX[i][j] = x[(int64_t)wrapp(o2 - 2 * PR + i, n2) * n1 + wrapp(o1 - 2 * PR + j, n1)];
    }
    // r task: column j of the r region, rows i0 .. i0 + RSEG - 1
    const bool rt = tid < RG * (RG / RSEG);
    const int rj = rt ? tid % RG : 0, ri0 = rt ? (tid / RG) * RSEG : 0;
    T f0v[RSEG];
#pragma unroll
    for (int q = 0; q < RSEG; ++q)
        f0v[q] = a.f0 ? a.f0[ch * a.plane + (int64_t)wrapp(o2 - PR + ri0 + q, n2) * n1 + wrapp(o1 - PR + rj, n1)]
                      : T(0);
    T racc[RSEG];
#pragma unroll
    for (int q = 0; q < RSEG; ++q) racc[q] = T(0);

    // multipliers of the x region for term k, prefetched one term ahead
    T vpre[XPT];
    auto load_v = [&](int k) {
        const T *v = a.v + (int64_t)k * n1 * n2;
#pragma unroll
        for (int t = 0; t < XPT; ++t) {
            const int e0 = tid + t * NTP, e = e0 < XG * XG ? e0 : XG * XG - 1;
            const int i = e / XG, j = e - i * XG;
            vpre[t] = v[(int64_t)wrapp(o2 - 2 * PR + i, n2) * n1 + wrapp(o1 - 2 * PR + j, n1)];
        }
    };
    load_v(0);
    for (int k = 0; k < a.m; ++k) {
        __syncthreads();  // previous term's sG / sU readers are done (and sX is staged)
        load_taps<T, NTP>(a, k, sU);
#pragma unroll
        for (int t = 0; t < XPT; ++t) {
            const int e = tid + t * NTP;
            if (e < XG * XG) {
                const int i = e / XG, j = e - i * XG;
                sG[i][j] = vpre[t] * sX[i][j];
            }
        }
        __syncthreads();
        if (k + 1 < a.m) load_v(k + 1);  // in flight during this term's stencil
        if (rt) {
            // r(i, j) += sum_{a,b} u(a - PR, b - PR) g(i + 2PR - a, j + 2PR - b)  (region indices)
            for (int b = 0; b < PW; ++b) {
                const int gj = rj + 2 * PR - b;
                T win[RSEG + 2 * PR];
#pragma unroll
                for (int t = 0; t < RSEG + 2 * PR; ++t) win[t] = sG[ri0 + t][gj];
#pragma unroll
                for (int aa = 0; aa < PW; ++aa) {
                    const T uv = sU[aa * PW + b];
#pragma unroll
                    for (int q = 0; q < RSEG; ++q) racc[q] = fma(uv, win[q + 2 * PR - aa], racc[q]);
                }
            }
        }
    }
    // r = H x - f0 on the r region; statistics over this tile's own pixels
    double st = 0.0;
    if (rt) {
#pragma unroll
        for (int q = 0; q < RSEG; ++q) {
            const T r = racc[q] - f0v[q];
            sR[ri0 + q][rj] = r;
            const int i = ri0 + q;
            const bool own = i >= PR && i < PR + PT && rj >= PR && rj < PR + PT && o2 - PR + i < n2 &&
                             o1 - PR + rj < n1;
            if (own) st += 0.5 * (double)r * (double)r;
        }
    }
    // s task: column j of the tile, rows i0 .. i0 + SSEG - 1
    const int sj = tid % PT, si0 = (tid / PT) * SSEG;
    T sacc[SSEG];
#pragma unroll
    for (int q = 0; q < SSEG; ++q) sacc[q] = T(0);
    T vv[SSEG], vn[SSEG];
    auto load_vo = [&](int k, T (&dst)[SSEG]) {
        const T *v = a.v + (int64_t)k * n1 * n2;
#pragma unroll
        for (int q = 0; q < SSEG; ++q) dst[q] = v[(int64_t)wrapp(o2 + si0 + q, n2) * n1 + wrapp(o1 + sj, n1)];
    };
    load_vo(0, vn);
    for (int k = 0; k < a.m; ++k) {
        __syncthreads();  // sR complete; previous term's sU readers done
        load_taps<T, NTP>(a, k, sU);
#pragma unroll
        for (int q = 0; q < SSEG; ++q) vv[q] = vn[q];
        __syncthreads();
        if (k + 1 < a.m) load_vo(k + 1, vn);
        T h[SSEG];
#pragma unroll
        for (int q = 0; q < SSEG; ++q) h[q] = T(0);
        // h(i, j) = sum_{a,b} u(a - PR, b - PR) r(i + a, j + b)  (r-region indices)
        for (int b = 0; b < PW; ++b) {
            T win[SSEG + 2 * PR];
#pragma unroll
            for (int t = 0; t < SSEG + 2 * PR; ++t) win[t] = sR[si0 + t][sj + b];
#pragma unroll
            for (int aa = 0; aa < PW; ++aa) {
                const T uv = sU[aa * PW + b];
#pragma unroll
                for (int q = 0; q < SSEG; ++q) h[q] = fma(uv, win[q + aa], h[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < SSEG; ++q) sacc[q] = fma(vv[q], h[q], sacc[q]);
    }
    T *s = a.s + ch * a.plane;
#pragma unroll
    for (int q = 0; q < SSEG; ++q) {
        const int gy = o2 + si0 + q, gx = o1 + sj;
        if (gy < n2 && gx < n1) s[(int64_t)gy * n1 + gx] = sacc[q];
    }
    if (a.slots) block_add1<T, NTP>(st, a.slots);
}

// One pass, one thread per output pixel: H x or H^T x (set-up and tests).
constexpr int NTS = 256;
template <typename T>
__global__ __launch_bounds__(NTS) void k_pc_single(PcArgs<T> a, int transpose)
{
    const int64_t p = (int64_t)blockIdx.x * NTS + threadIdx.x;
    const int n1 = a.n1, n2 = a.n2;
    if (p >= (int64_t)n1 * n2) return;
    const int i2 = (int)(p / n1), i1 = (int)(p - (int64_t)i2 * n1);
    const int64_t ch = blockIdx.y;
    const T *x = a.x + ch * a.plane;
    const int R = a.R, W = 2 * R + 1;
    T acc = T(0);
    for (int k = 0; k < a.m; ++k) {
        const T *u = a.u + (int64_t)k * W * W;
        const T *v = a.v + (int64_t)k * n1 * n2;
        T hk = T(0);
        for (int d2 = -R; d2 <= R; ++d2) {
            // H: u(d) v(p - d) x(p - d);  H^T: u(d) x(p + d), weighted by v(p) after the sum
            const int y2 = wrapp(transpose ? i2 + d2 : i2 - d2, n2);
            for (int d1 = -R; d1 <= R; ++d1) {
                const int y1 = wrapp(transpose ? i1 + d1 : i1 - d1, n1);
                const int64_t q = (int64_t)y2 * n1 + y1;
                const T g = transpose ? x[q] : v[q] * x[q];
                hk = fma(u[(d2 + R) * W + (d1 + R)], g, hk);
            }
        }
        acc += transpose ? v[p] * hk : hk;
    }
    a.s[ch * a.plane + p] = acc;
}

}  // namespace

template <typename T>
hipError_t launch_pcblur(const PcArgs<T> &a, hipStream_t s)
{
    dim3 grid((a.n1 + PT - 1) / PT, (a.n2 + PT - 1) / PT, a.C);
    // few tiles: twice the threads per tile so that every SIMD holds two waves
    if ((int64_t)grid.x * grid.y * grid.z < 512)
        hipLaunchKernelGGL((k_pcblur<T, PcLarge>), grid, dim3(PcLarge::nt), 0, s, a);
    else
        hipLaunchKernelGGL((k_pcblur<T, PcSmall>), grid, dim3(PcSmall::nt), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pc_single(const PcArgs<T> &a, int transpose, hipStream_t s)
{
    const int64_t N = (int64_t)a.n1 * a.n2;
    dim3 grid((unsigned)((N + NTS - 1) / NTS), a.C);
    hipLaunchKernelGGL(k_pc_single<T>, grid, dim3(NTS), 0, s, a, transpose);
    return hipGetLastError();
}

template hipError_t launch_pcblur<float>(const PcArgs<float> &, hipStream_t);
template hipError_t launch_pcblur<double>(const PcArgs<double> &, hipStream_t);
template hipError_t launch_pc_single<float>(const PcArgs<float> &, int, hipStream_t);
template hipError_t launch_pc_single<double>(const PcArgs<double> &, int, hipStream_t);

}  // namespace pd
