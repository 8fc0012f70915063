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
// Fine levels run one LDS-tiled kernel per level; all levels whose
// approximation fits one workgroup's LDS run in a single "coarse" kernel that
// also starts the next iteration's synthesis.  Each workgroup first issues
// all of its global loads (so their latencies overlap), then filters from LDS
// with register blocking (each thread produces several neighbouring outputs
// from one window of inputs held in registers).  FP64 statistics use one
// atomic per workgroup.  Filters are zero-padded to 12 taps so any even
// length <= 12 runs the same code.
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <mutex>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "pd_kernels.h"

namespace pd {

constexpr int NT = 256;  // threads per workgroup (4 wave64)

// a mod n for any a; the in-range case costs two compares
__device__ __forceinline__ int wrap(int a, int n)
{
    if (a >= 0 && a < n) return a;
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Cross-lane sums on the DPP network (no LDS round trip).  dpp_row_sum:
// every lane of a 16-lane row receives the row's sum, added pairwise as
// (lane ^ 1), (lane ^ 2), mirror in 8, mirror in 16, so all lanes of the row
// hold the same bits.  wave_sum: the sum of the four row sums, uniform.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename T>
__device__ __forceinline__ T dpp_row_sum(T x)
{
    if constexpr (sizeof(T) == 4) {
        x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
        x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
        x += dpp_f<0x141>(x);  // row_half_mirror
        x += dpp_f<0x140>(x);  // row_mirror
    } else {
        x += dpp_d<0xB1>(x);
        x += dpp_d<0x4E>(x);
        x += dpp_d<0x141>(x);
        x += dpp_d<0x140>(x);
    }
    return x;
}
__device__ __forceinline__ double lane_d(double x, int l)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double x)
{
    x = dpp_row_sum(x);
    return (lane_d(x, 0) + lane_d(x, 16)) + (lane_d(x, 32) + lane_d(x, 48));
}

// x as a wave-uniform (scalar register) value; used so that selects between
// argument-block entries do not become per-lane loads from the argument block.
template <typename T>
__device__ __forceinline__ T uniform(T x)
{
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
    } else {
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
        const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
}

// Block-wide sums of NV doubles; thread q adds sum q to row q of the
// [NV][PD_NSLOT] slot array at a slot chosen by the block index, so that
// concurrent workgroups rarely hit the same address.  Contains a barrier.
template <int NV, int NTH>
__device__ void block_slot_add(double (&v)[NV], double *slots)
{
    __shared__ double red[NV][NTH / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double a = wave_sum(v[q]);
        if (lane == 0) red[q][wv] = a;
    }
    __syncthreads();
    static_assert(NV <= 4 && NTH / 64 <= 16, "one DPP row per sum");
    if (wv == 0) {  // lane = 16 q + k: row q sums the NTH/64 wave partials of sum q
        const int q = lane >> 4, k = lane & 15;
        const double a = dpp_row_sum((q < NV && k < NTH / 64) ? red[q < NV ? q : 0][k] : 0.0);
        const unsigned blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        if (q < NV && k == 0) atomicAdd(slots + q * PD_NSLOT + (blk % PD_NSLOT), a);
    }
}

// y = a + beta (a - b), the momentum step, as one explicit fused multiply-add, so
// that every kernel forming a y from the same two iterates gets the same bits.
template <typename T>
__device__ __forceinline__ T momentum(T a, T b, T beta)
{
    return fma(beta, a - b, a);
}

// A product rounded on its own (never fused into a later add): the joint prox's
// z feeds both its store and, in the coarse kernel, the next y, which must be
// formed from the stored (rounded) z as a later launch would form it.
__device__ __forceinline__ float mul_rn(float a, float b)
{
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double mul_rn(double a, double b)
{
#pragma clang fp contract(off)
    return a * b;
}

// Soft threshold S_t(v) = sign(v) max(|v| - t, 0), zero on |v| <= t.
template <typename T>
__device__ __forceinline__ T soft(T v, T t)
{
    T a = fabs(v) - t;
    return a > T(0) ? copysign(a, v) : T(0);
}

// Gradient step + prox + momentum bookkeeping for one coefficient of one
// channel (scalar weights).  Returns z; accumulates w|y| and (z-y)^2.
// v = y - tau g as one explicit fused multiply-add (every prox of every
// kernel forms it the same way, so the fused and the split paths agree bit
// for bit).
template <typename T>
__device__ __forceinline__ T grad_step(T y, T g, T tau)
{
    return fma(-tau, g, y);
}

template <typename T>
__device__ __forceinline__ T prox1(T y, T g, T tau, T w, double (&st)[2], bool &bad)
{
    T v = grad_step(y, g, tau);
    T z = soft(v, tau * w);
    bad |= !isfinite(v);
    st[0] += (double)w * fabs((double)y);
    st[1] += ((double)z - (double)y) * ((double)z - (double)y);
    return z;
}

// ===========================================================================
// Synthesis of one fine level (Section 2.1 expansion, x2 then x1):
//   fine[n] = sum_l h[n-2l] lo[l] + g[n-2l] hi[l];
// for output n = 2p + par the low-pass terms are l = p-5+j with tap
// h[par+10-2j] and the high-pass terms l = p+j with tap g[par-2j], j = 0..5.
// A workgroup produces a 32 x 32 fine tile from 16 x 16 (+10 halo) of each band.
// ===========================================================================
constexpr int SP = 16;          // coarse tile per band
constexpr int SR = SP + 10;     // with halo
constexpr int SF = 2 * SP;      // fine tile
static_assert((2 * SR) % (NT / 64) == 0, "synthesis load rows per wave");

template <typename T>
__device__ __forceinline__ void synth_body(const SynthArgs<T> &a, const Live<T> &lv, int bx, int by, int bz)
{
    __shared__ T sB[4][SR][SR + 1];   // LL, HL (hi x1), LH (hi x2), HH
    __shared__ T sLH[2][SF][SR + 1];  // after x2 synthesis: low / high along x1
    const int M1c = a.M1c, M2c = a.M2c;
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int64_t ch = bz;
    const int p01 = bx * SP, p02 = by * SP;
    const T *zc = lv.zc + ch * a.plane;
    const T *zp = lv.zp + ch * a.plane;
    const T *apx = a.apx ? a.apx + ch * a.apx_plane : nullptr;
    const int tid = threadIdx.x;

    // load: wave-row R < 26 covers the top bands (LL | HL) of coarse row R,
    // R >= 26 the bottom bands (LH | HH); lanes 0..25 the low-x1 band, 26..51
    // the high-x1 band.  Column offsets are per lane, row bases per wave-row.
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool lok = lane < 2 * SR;
    const bool hi1 = lane >= SR;
    const int lc_ = min(hi1 ? lane - SR : lane, SR - 1);  // lanes >= 2 SR read a neighbour, unused
    const int q1 = wrap(p01 - 5 + lc_, M1c);
    const int col = q1 + (hi1 ? M1c : 0);
    constexpr int RPW = (2 * SR) / (NT / 64);  // 13 wave-rows per wave
    // Every load is issued unconditionally (no data-dependent branch between
    // a load and its use): the approximation band reads apx twice when given.
    T va[RPW], vb[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int R = wv + i * (NT / 64);
        const bool bottom = R >= SR;
        const int r = bottom ? R - SR : R;
        const int q2 = wrap(p02 - 5 + r, M2c);
        const bool from_apx = !bottom && !hi1 && apx;
        const int64_t idx = from_apx ? (int64_t)q2 * M1c + q1
                                     : (int64_t)(q2 + (bottom ? M2c : 0)) * a.pitch + col;
        va[i] = (from_apx ? apx : zc)[idx];
        vb[i] = (from_apx ? apx : zp)[idx];
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int R = wv + i * (NT / 64);
        const bool bottom = R >= SR;
        const int r = bottom ? R - SR : R;
        if (lok) sB[(hi1 ? 1 : 0) + (bottom ? 2 : 0)][r][lc_] = momentum(va[i], vb[i], lv.beta);
    }
    __syncthreads();

    // along x2: task = (band, coarse column c, block of 4 output pairs)
    for (int t = tid; t < 2 * SR * (SP / 4); t += NT) {
        int band = t / (SR * (SP / 4)), rem = t - band * SR * (SP / 4);
        int blk = rem / SR, c = rem - blk * SR;
        const int bl = band, bh = band + 2;
        T lo[9], hi[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            lo[j] = sB[bl][4 * blk + j][c];
            hi[j] = sB[bh][4 * blk + 5 + j][c];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    acc = fma(a.f.h[par + 10 - 2 * j], lo[q + j], acc);
                    acc = fma(a.f.g[par - 2 * j + 10], hi[q + j], acc);
                }
                sLH[band][8 * blk + 2 * q + par][c] = acc;
            }
        }
    }
    __syncthreads();

    // along x1: task = (fine row f, block of 2 output pairs)
    T *out = a.out + ch * a.out_plane;
    for (int t = tid; t < SF * (SP / 2); t += NT) {
        int f = t / (SP / 2), blk = t - f * (SP / 2);
        T lo[7], hi[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            lo[j] = sLH[0][f][2 * blk + j];
            hi[j] = sLH[1][f][2 * blk + 5 + j];
        }
        const int o2 = 2 * p02 + f;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    acc = fma(a.f.h[par + 10 - 2 * j], lo[q + j], acc);
                    acc = fma(a.f.g[par - 2 * j + 10], hi[q + j], acc);
                }
                const int o1 = 2 * p01 + 4 * blk + 2 * q + par;
                if (o2 < M2 && o1 < M1) out[(int64_t)o2 * a.out_pitch + o1] = acc;
            }
        }
    }
}

// ===========================================================================
// Two synthesis levels in one launch: the coarser level U = D + 1 and the finer
// level D.  A workgroup produces the same 32 x 32 tile of level D's output as
// synth_body, computing the 26 x 26 part of level D's approximation band it
// reads (the output of level U) from a 24 x 24 region of level U's bands in
// LDS instead of reading it from memory.  Every output is formed by the same
// sums in the same order as the two single-level launches, so the results are
// the same bits; the saving is one launch and one round trip to memory.
// ===========================================================================
constexpr int UQ = SP / 2 + 6;   // level-U output pairs per axis (14): outputs [p0 - 6, p0 + 22)
constexpr int UR = UQ + 10;      // level-U band positions per axis (24)
constexpr int UO = 2 * UQ;       // level-U outputs per axis (28)
constexpr int VQ = UR / 2;       // level-V output pairs per axis (12): level-U band positions [P0 - 5, P0 + 19)
constexpr int VR = VQ + 10;      // level-V band positions per axis (22)

// One synthesis level over a region in LDS: the bands src[b] (b = LL, HL, LH,
// HH; NQ + 10 positions per axis, from 5 before the first output pair) give
// 2 NQ outputs per axis, along x2 into mid, then along x1; output (r, c) goes
// to dst[r - OFF][c - OFF] when both lie in [0, ND).  Same formula and order
// as synth_body.
template <typename T, int NQ, int ND, int OFF, int NTS = NT>
__device__ __forceinline__ void syn_region(const Filt<T> &f, T (*src)[NQ + 10][NQ + 11], T (*mid)[2 * NQ][NQ + 11],
                                           T (*dst)[ND + 1])
{
    constexpr int NR = NQ + 10;
    const int tid = threadIdx.x;
    // along x2: task = (band pair, column c, output pair q)
    for (int t = tid; t < 2 * NR * NQ; t += NTS) {
        const int band = t / (NR * NQ), rem = t - band * (NR * NQ), q = rem / NR, c = rem - q * NR;
        T lo[6], hi[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            lo[j] = src[band][q + j][c];
            hi[j] = src[band + 2][q + 5 + j][c];
        }
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                acc = fma(f.h[par + 10 - 2 * j], lo[j], acc);
                acc = fma(f.g[par - 2 * j + 10], hi[j], acc);
            }
            mid[band][2 * q + par][c] = acc;
        }
    }
    __syncthreads();
    // along x1
    for (int t = tid; t < 2 * NQ * NQ; t += NTS) {
        const int r = t / NQ, q = t - r * NQ;
        T lo[6], hi[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            lo[j] = mid[0][r][q + j];
            hi[j] = mid[1][r][q + 5 + j];
        }
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                acc = fma(f.h[par + 10 - 2 * j], lo[j], acc);
                acc = fma(f.g[par - 2 * j + 10], hi[j], acc);
            }
            const int rr = r - OFF, cc = 2 * q + par - OFF;
            if (rr >= 0 && rr < ND && cc >= 0 && cc < ND) dst[rr][cc] = acc;
        }
    }
    __syncthreads();
}

// Level D of a fused synthesis: the passes of synth_body over sB (its bands
// at p0 - 5 .. p0 + 20), output tile at fine position 2 p0.
template <typename T, int NTS = NT>
__device__ __forceinline__ void syn_level_d(const SynthArgs<T> &d, T (*sB)[SR][SR + 1], T (*sLH)[SF][SR + 1], int64_t ch,
                                            int p01, int p02)
{
    const int tid = threadIdx.x;
    for (int t = tid; t < 2 * SR * (SP / 4); t += NTS) {
        int band = t / (SR * (SP / 4)), rem = t - band * SR * (SP / 4);
        int blk = rem / SR, c = rem - blk * SR;
        const int bl = band, bh = band + 2;
        T lo[9], hi[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            lo[j] = sB[bl][4 * blk + j][c];
            hi[j] = sB[bh][4 * blk + 5 + j][c];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    acc = fma(d.f.h[par + 10 - 2 * j], lo[q + j], acc);
                    acc = fma(d.f.g[par - 2 * j + 10], hi[q + j], acc);
                }
                sLH[band][8 * blk + 2 * q + par][c] = acc;
            }
        }
    }
    __syncthreads();
    T *out = d.out + ch * d.out_plane;
    const int M1 = 2 * d.M1c, M2 = 2 * d.M2c;
    for (int t = tid; t < SF * (SP / 2); t += NTS) {
        int f = t / (SP / 2), blk = t - f * (SP / 2);
        T lo[7], hi[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            lo[j] = sLH[0][f][2 * blk + j];
            hi[j] = sLH[1][f][2 * blk + 5 + j];
        }
        const int o2 = 2 * p02 + f;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                T acc = T(0);
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    acc = fma(d.f.h[par + 10 - 2 * j], lo[q + j], acc);
                    acc = fma(d.f.g[par - 2 * j + 10], hi[q + j], acc);
                }
                const int o1 = 2 * p01 + 4 * blk + 2 * q + par;
                if (o2 < M2 && o1 < M1) out[(int64_t)o2 * d.out_pitch + o1] = acc;
            }
        }
    }
}

// Index of a state-plane band value: band b (0 LL, 1 HL, 2 LH, 3 HH) of a
// level with M1 x M2 bands, at wrapped band position (q2, q1).
__device__ __forceinline__ int64_t band_at(int b, int q2, int q1, int M1, int M2, int pitch)
{
    return (int64_t)(q2 + (b >= 2 ? M2 : 0)) * pitch + q1 + ((b & 1) ? M1 : 0);
}

template <typename T>
__device__ __forceinline__ void synth2_body(const SynthArgs<T> &d, const SynthArgs<T> &u, const Live<T> &lv, int bx,
                                            int by, int bz)
{
    __shared__ T sU[4][UR][UR + 1];   // level U: LL, HL, LH, HH
    __shared__ T sUL[2][UO][UR + 1];  // level U after x2: low / high along x1
    __shared__ T sB[4][SR][SR + 1];   // level D: LL (= level U's output), HL, LH, HH
    __shared__ T sLH[2][SF][SR + 1];  // level D after x2
    const int64_t ch = bz;
    const int p01 = bx * SP, p02 = by * SP;  // level-D coarse tile origin
    const int P01 = p01 / 2 - 3, P02 = p02 / 2 - 3;  // level-U output pair origin
    const T *zc = lv.zc + ch * d.plane;
    const T *zp = lv.zp + ch * d.plane;
    const T *apx = u.apx ? u.apx + ch * u.apx_plane : nullptr;
    const int tid = threadIdx.x;
    const int M1u = u.M1c, M2u = u.M2c, M1d = d.M1c, M2d = d.M2c;

    // every load up front: the four level-U bands (24 x 24 from position P0 - 5) and the three
    // level-D detail bands (26 x 26 from position p0 - 5); y = z(i-1) + beta (z(i-1) - z(i-2))
    constexpr int NU = 4 * UR * UR, ND = 3 * SR * SR, NL = (NU + ND + NT - 1) / NT;
    T va[NL], vb[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        int e = tid + k * NT;
        e = e < NU + ND ? e : 0;  // past the end: an in-range duplicate, unused
        int64_t idx;
        bool from_apx = false;
        if (e < NU) {
            const int b = e / (UR * UR), rem = e - b * (UR * UR), r = rem / UR, c = rem - r * UR;
            const int q2 = wrap(P02 - 5 + r, M2u), q1 = wrap(P01 - 5 + c, M1u);
            from_apx = b == 0 && apx;
            idx = from_apx ? (int64_t)q2 * M1u + q1 : band_at(b, q2, q1, M1u, M2u, d.pitch);
        } else {
            const int e2 = e - NU, b = 1 + e2 / (SR * SR), rem = e2 - (b - 1) * (SR * SR), r = rem / SR,
                      c = rem - r * SR;
            const int q2 = wrap(p02 - 5 + r, M2d), q1 = wrap(p01 - 5 + c, M1d);
            idx = band_at(b, q2, q1, M1d, M2d, d.pitch);
        }
        va[k] = (from_apx ? apx : zc)[idx];
        vb[k] = (from_apx ? apx : zp)[idx];
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int e = tid + k * NT;
        if (e >= NU + ND) continue;
        const T y = momentum(va[k], vb[k], lv.beta);
        if (e < NU) {
            const int b = e / (UR * UR), rem = e - b * (UR * UR), r = rem / UR, c = rem - r * UR;
            sU[b][r][c] = y;
        } else {
            const int e2 = e - NU, b = 1 + e2 / (SR * SR), rem = e2 - (b - 1) * (SR * SR), r = rem / SR,
                      c = rem - r * SR;
            sB[b][r][c] = y;
        }
    }
    __syncthreads();
    // level U into the approximation band of level D (output n <-> sB row / column n - (p0 - 5))
    syn_region<T, UQ, SR, 1>(d.f, sU, sUL, sB[0]);  // (u's filter bank is d's)
    syn_level_d<T>(d, sB, sLH, ch, p01, p02);
}

// ===========================================================================
// Three synthesis levels in one launch: V = D + 2, U = D + 1 and D.  As
// synth2_body, with the 24 x 24 part of level U's approximation band that the
// U stage reads computed from a 22 x 22 region of level V's bands in LDS
// (level V's outputs [P0 - 5, P0 + 19) per axis, exactly that region).  Same
// sums in the same order as the single-level launches: the same bits.
// ===========================================================================
template <typename T, int NTS = NT>
__device__ __forceinline__ void synth3_body(const SynthArgs<T> &d, const SynthArgs<T> &u, const SynthArgs<T> &v,
                                            const Live<T> &lv, int bx, int by, int bz)
{
    __shared__ T sV[4][VR][VR + 1];   // level V: LL, HL, LH, HH
    __shared__ T sVL[2][UR][VR + 1];  // level V after x2
    __shared__ T sU[4][UR][UR + 1];   // level U: LL (= level V's output), HL, LH, HH
    __shared__ T sUL[2][UO][UR + 1];
    __shared__ T sB[4][SR][SR + 1];   // level D: LL (= level U's output), HL, LH, HH
    __shared__ T sLH[2][SF][SR + 1];
    const int64_t ch = bz;
    const int p01 = bx * SP, p02 = by * SP;          // level-D coarse tile origin
    const int P01 = p01 / 2 - 3, P02 = p02 / 2 - 3;  // level-U output pair origin
    const int R01 = (P01 - 5) / 2 - 5, R02 = (P02 - 5) / 2 - 5;  // level-V band region origin (P0 - 5 is even)
    const T *zc = lv.zc + ch * d.plane;
    const T *zp = lv.zp + ch * d.plane;
    const T *apx = v.apx ? v.apx + ch * v.apx_plane : nullptr;
    const int tid = threadIdx.x;
    const int M1v = v.M1c, M2v = v.M2c, M1u = u.M1c, M2u = u.M2c, M1d = d.M1c, M2d = d.M2c;

    // every load up front: level V's four bands (22 x 22), level U's and level D's detail bands
    constexpr int NV = 4 * VR * VR, NU = 3 * UR * UR, ND = 3 * SR * SR, NA = NV + NU + ND;
    constexpr int NL = (NA + NTS - 1) / NTS;
    T va[NL], vb[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        int e = tid + k * NTS;
        e = e < NA ? e : 0;  // past the end: an in-range duplicate, unused
        int64_t idx;
        bool from_apx = false;
        if (e < NV) {
            const int b = e / (VR * VR), rem = e - b * (VR * VR), r = rem / VR, c = rem - r * VR;
            const int q2 = wrap(R02 + r, M2v), q1 = wrap(R01 + c, M1v);
            from_apx = b == 0 && apx;
            idx = from_apx ? (int64_t)q2 * M1v + q1 : band_at(b, q2, q1, M1v, M2v, d.pitch);
        } else if (e < NV + NU) {
            const int e2 = e - NV, b = 1 + e2 / (UR * UR), rem = e2 - (b - 1) * (UR * UR), r = rem / UR,
                      c = rem - r * UR;
            idx = band_at(b, wrap(P02 - 5 + r, M2u), wrap(P01 - 5 + c, M1u), M1u, M2u, d.pitch);
        } else {
            const int e2 = e - NV - NU, b = 1 + e2 / (SR * SR), rem = e2 - (b - 1) * (SR * SR), r = rem / SR,
                      c = rem - r * SR;
            idx = band_at(b, wrap(p02 - 5 + r, M2d), wrap(p01 - 5 + c, M1d), M1d, M2d, d.pitch);
        }
        va[k] = (from_apx ? apx : zc)[idx];
        vb[k] = (from_apx ? apx : zp)[idx];
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int e = tid + k * NTS;
        if (e >= NA) continue;
        const T y = momentum(va[k], vb[k], lv.beta);
        if (e < NV) {
            const int b = e / (VR * VR), rem = e - b * (VR * VR), r = rem / VR, c = rem - r * VR;
            sV[b][r][c] = y;
        } else if (e < NV + NU) {
            const int e2 = e - NV, b = 1 + e2 / (UR * UR), rem = e2 - (b - 1) * (UR * UR), r = rem / UR,
                      c = rem - r * UR;
            sU[b][r][c] = y;
        } else {
            const int e2 = e - NV - NU, b = 1 + e2 / (SR * SR), rem = e2 - (b - 1) * (SR * SR), r = rem / SR,
                      c = rem - r * SR;
            sB[b][r][c] = y;
        }
    }
    __syncthreads();
    // (every level's arguments carry the same filter bank: d's is used throughout)
    syn_region<T, VQ, UR, 0, NTS>(d.f, sV, sVL, sU[0]);  // level V into level U's approximation band
    syn_region<T, UQ, SR, 1, NTS>(d.f, sU, sUL, sB[0]);  // level U into level D's approximation band
    syn_level_d<T, NTS>(d, sB, sLH, ch, p01, p02);
}

// ===========================================================================
// Analysis of one fine level (Section 2.1):
//   lo[l] = sum_{k=0}^{11} h[k] in[2l+k],  hi[l] = sum_{k=-10}^{1} g[k] in[2l+k]
// along x1 then x2.  A workgroup produces a 16 x 16 tile of each band from a
// 52 x 52 fine region; the detail bands (and, at the coarsest level, the
// approximation band) go through the fused gradient step + prox + momentum,
// or are stored plainly.
// ===========================================================================
constexpr int TC = 16;
constexpr int AR = 2 * TC + 20;  // fine region incl. halo
static_assert(AR % (NT / 64) == 0 && AR <= 64, "analysis load rows per wave");

// NCH = 0: one channel with scalar (or per-coefficient) weights; NCH >= 1:
// the joint colour prox over NCH channels handled by one workgroup.
template <typename T, int NCH>
__device__ __forceinline__ void analysis_body(const AnalysisArgs<T> &a, const Live<T> &lv, int bx, int by, int bz)
{
    constexpr bool JOINT = NCH > 0;
    constexpr int NC = JOINT ? NCH : 1;
    // LDS layouts without bank conflicts: the x1 pass reads 16-byte runs of
    // sIn rows with the lanes of a 16-lane group on consecutive rows (pitch 52 =
    // 13 x 16 bytes: each row starts on a different 16-byte bank group), and
    // writes its four outputs per row as one 16-byte store; the x2 pass reads
    // sRow columns with four row blocks per wave, which a pitch of 20 puts on
    // disjoint banks (a block's rows are 4 x 20 = 80 values = 16 banks apart)
    __shared__ __attribute__((aligned(16))) T sIn[AR][AR];
    __shared__ __attribute__((aligned(16))) T sRow[2][AR][TC + 4];  // low / high along x1
    const int M1c = a.M1c, M2c = a.M2c;
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int c01 = bx * TC, c02 = by * TC;
    const int tid = threadIdx.x;
    const ProxArgs<T> &p = a.p;
    const int ch0 = JOINT ? 0 : bz;

    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool lok = lane < AR;
    const int qc = lok ? wrap(2 * c01 - 10 + lane, M1) : 0;
    // column-pass task of this thread: (src band along x1, coarse column, 2 rows)
    const int src = tid / (TC * (TC / 2));
    const int rem = tid - src * (TC * (TC / 2));
    const int rblk = rem / TC, l1 = rem - rblk * TC;
    T res[NC][4];  // [ch][ (h, g) x 2 rows ]

    // outputs of this thread (band, row) in its column, and the prox operands
    // for them: loaded first (clamped, unconditional) so that they arrive
    // while the tile is transformed.  z(i) is written in place of z(i-2) only
    // at the thread's own positions, after these reads.
    const int g1 = c01 + l1;
    const bool prox = a.mode == MODE_PROX;
    T zcr[NC][4], zpr[NC][4], wr[4];
    int64_t idxs[4];
    bool valid[4], toapx[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int q = o >> 1, hx2 = o & 1;
        const int b = src + 2 * hx2;  // bit 0: high along x1, bit 1: high along x2
        const int g2 = c02 + 2 * rblk + q;
        valid[o] = g2 < M2c && g1 < M1c;
        toapx[o] = b == 0 && !a.last;
        idxs[o] = (int64_t)(g2 + (hx2 ? M2c : 0)) * p.pitch + g1 + (src ? M1c : 0);
        const bool use = valid[o] && !toapx[o] && prox;
        // unused loads read an in-range neighbour (spread addresses), of the
        // state in prox mode, else of the input row this lane loads anyway
        const int64_t near = prox ? (int64_t)((g2 < M2c ? g2 : M2c - 1) + (hx2 ? M2c : 0)) * p.pitch +
                                        (g1 < M1c ? g1 : M1c - 1) + (src ? M1c : 0)
                                  : (int64_t)wrap(2 * c02, M2) * a.in_pitch + qc;
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
            const int64_t ci = prox ? (int64_t)(ch0 + cc) * p.plane + near : near;
            const T u = (prox ? lv.zc : a.in)[ci];
            const T v = (prox ? lv.zp : a.in)[ci];
            zcr[cc][o] = use ? u : T(0);
            zpr[cc][o] = use ? v : T(0);
        }
        const bool usew = prox && p.wmap;
        const T wv_ = (usew ? p.wmap : a.in)[usew ? (int64_t)ch0 * p.plane + near : near];
        wr[o] = use && usew ? wv_ : T(0);
    }

    // load every channel's tile at once: lane = fine column (52 of 64 lanes), wave = fine rows
    constexpr int RPW = AR / (NT / 64);  // 13
    T v[NC][RPW];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
        const T *in = a.in + (int64_t)(ch0 + cc) * a.in_plane;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + i * (NT / 64);
            const T *rowp = in + (int64_t)wrap(2 * c02 - 10 + r, M2) * a.in_pitch;
            v[cc][i] = rowp[qc];
        }
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
        if (cc > 0) __syncthreads();  // previous channel's passes are done
#pragma unroll
        for (int i = 0; i < RPW; ++i)
            if (lok) sIn[wv + i * (NT / 64)][lane] = v[cc][i];
        __syncthreads();
        // along x1: task = (fine row r, block of 4 coarse columns), lanes on rows
        for (int t = tid; t < AR * (TC / 4); t += NT) {
            const int blk = t / AR, r = t - blk * AR;
            T x[28];
#pragma unroll
            for (int j = 0; j < 28; ++j) x[j] = sIn[r][8 * blk + j];
            using V4 = T __attribute__((ext_vector_type(4)));
            V4 lo4, hi4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T lo = T(0), hi = T(0);
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    lo = fma(a.f.h[m], x[2 * q + m + 10], lo);
                    hi = fma(a.f.g[m], x[2 * q + m], hi);
                }
                lo4[q] = lo;
                hi4[q] = hi;
            }
            *reinterpret_cast<V4 *>(&sRow[0][r][4 * blk]) = lo4;
            *reinterpret_cast<V4 *>(&sRow[1][r][4 * blk]) = hi4;
        }
        __syncthreads();
        // along x2: 2 coarse rows of both x2 filters for one column of one band
        {
            T x[24];
#pragma unroll
            for (int j = 0; j < 24; ++j) x[j] = sRow[src][4 * rblk + j][l1];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                T lo = T(0), hi = T(0);
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    lo = fma(a.f.h[m], x[2 * q + m + 10], lo);
                    hi = fma(a.f.g[m], x[2 * q + m], hi);
                }
                res[cc][2 * q + 0] = lo;
                res[cc][2 * q + 1] = hi;
            }
        }
    }

    // epilogue: stores and prox
    double st[2] = {0.0, 0.0};
    bool bad = false;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int q = o >> 1, hx2 = o & 1;
        const int b = src + 2 * hx2;
        if (!valid[o]) continue;
        if (toapx[o]) {
            const int g2 = c02 + 2 * rblk + q;
#pragma unroll
            for (int cc = 0; cc < NC; ++cc)
                a.apx_out[(int64_t)(ch0 + cc) * a.apx_plane + (int64_t)g2 * M1c + g1] = res[cc][2 * q + hx2];
            continue;
        }
        const int64_t idx = idxs[o];
        if (!prox) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) lv.zn[(int64_t)(ch0 + cc) * p.plane + idx] = res[cc][2 * q + hx2];
            continue;
        }
        // band weight: a select between two uniform table entries (a per-lane
        // index into the argument block would be a vector load per lane)
        const T wband = b == 0 ? uniform(p.wlev[0]) : uniform(p.wlev[a.band_detail]);
        if (!JOINT) {
            T w = p.wmap ? wr[o] : wband;
            T y = momentum(zcr[0][o], zpr[0][o], lv.beta);
            const T z = prox1(y, res[0][2 * q + hx2], p.tau, w, st, bad);
            lv.zn[(int64_t)ch0 * p.plane + idx] = z;
            if (p.zsave) p.zsave[(int64_t)ch0 * p.plane + idx] = z;
        } else {
            T yv[NC], vv[NC];
            T nv = T(0);
            double ny = 0.0;
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                yv[cc] = momentum(zcr[cc][o], zpr[cc][o], lv.beta);
                vv[cc] = grad_step(yv[cc], res[cc][2 * q + hx2], p.tau);
                nv = fma(vv[cc], vv[cc], nv);
                ny += (double)yv[cc] * (double)yv[cc];
            }
            T w = wband;
            T nrm = sqrt(nv);
            T sc = nrm > T(0) ? T(1) - p.tau * w / nrm : T(0);
            sc = sc > T(0) ? sc : T(0);
            bad |= !isfinite(nrm);
            st[0] += (double)w * sqrt(ny);
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) {
                T z = mul_rn(vv[cc], sc);
                lv.zn[(int64_t)cc * p.plane + idx] = z;
                if (p.zsave) p.zsave[(int64_t)cc * p.plane + idx] = z;
                st[1] += ((double)z - (double)yv[cc]) * ((double)z - (double)yv[cc]);
            }
        }
    }
    if (a.mode == MODE_PROX) {
        if (lv.slots) block_slot_add<2, NT>(st, lv.slots + PD_NSLOT);
        if (bad) atomicOr(p.flag, 1);
    }
}

// ===========================================================================
// Two analysis levels in one launch (gradient step + prox or plain mode, one
// channel per tile set): levels D and E = D + 1.  A workgroup owns a 16 x 16 tile of
// level D's bands and the 8 x 8 tile of level E's bands below it.  From one
// 82 x 82 region of level D's input in LDS it computes (i) level D's detail
// bands on the owned tile, exactly as analysis_body does, and (ii) level D's
// approximation band on the 36 x 36 region that level E's tile reads (the
// owned 16 x 16 and a 10-wide ring, which neighbouring workgroups own too),
// then level E from that region.  Every value is the same sum in the same
// order as in the single-level launches, so the outputs carry the same bits;
// level D's approximation band never leaves LDS.
// ===========================================================================
constexpr int TE = TC / 2;          // level E tile
constexpr int LR = 2 * TE + 20;     // level D approximation region (36)
constexpr int BR = 2 * LR + 10;     // level D input region (82)
constexpr int BRP = BR + 2;         // its LDS pitch

template <typename T, int NTS>
__device__ __forceinline__ void analysis2_body(const AnalysisArgs<T> &a, const AnalysisArgs<T> &e, const Live<T> &lv,
                                               int bx, int by, int bz)
{
    static_assert(NTS >= NT && NTS % 64 == 0, "the epilogue uses the first NT threads");
    __shared__ __attribute__((aligned(16))) T sIn[BR][BRP];
    __shared__ __attribute__((aligned(16))) T sRow[2][AR][TC + 4];  // level D details, as analysis_body
    __shared__ T sLo[BR][LR + 1];                                   // level D low-pass along x1
    __shared__ T sLL[LR][LR + 1];                                   // level D approximation region
    __shared__ T sRowE[2][LR][TE + 1];                              // level E along x1
    const int M1c = a.M1c, M2c = a.M2c, M1 = 2 * M1c, M2 = 2 * M2c;
    const int M1e = e.M1c, M2e = e.M2c;
    const int c01 = bx * TC, c02 = by * TC;  // level D tile origin
    const int e01 = bx * TE, e02 = by * TE;  // level E tile origin
    const int tid = threadIdx.x;
    const ProxArgs<T> &p = a.p;
    const bool prox = a.mode == MODE_PROX;
    const int64_t ch = bz;
    const T *in = a.in + ch * a.in_plane;

    // level D outputs of this thread (analysis_body's mapping) and the level E
    // output (band src + 2 hx2, row er, column ec); prox operands loaded first
    const int src = tid / (TC * (TC / 2));
    const int rem = tid - src * (TC * (TC / 2));
    const int rblk = rem / TC, l1 = rem - rblk * TC;
    const int g1 = c01 + l1;
    const int esrc = tid >> 7, ehx2 = (tid >> 6) & 1, er = (tid >> 3) & 7, ec = tid & 7;
    const int eg1 = e01 + ec, eg2 = e02 + er;
    T zcr[5], zpr[5], wr[5];
    int64_t idxs[5];
    bool valid[5], use[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        int64_t idx, near;
        if (o < 4) {
            const int q = o >> 1, hx2 = o & 1;
            const int g2 = c02 + 2 * rblk + q;
            valid[o] = g2 < M2c && g1 < M1c;
            use[o] = tid < NT && valid[o] && src + 2 * hx2 != 0;  // level D's approximation stays in LDS
            idx = (int64_t)(g2 + (hx2 ? M2c : 0)) * p.pitch + g1 + (src ? M1c : 0);
            near = (int64_t)((g2 < M2c ? g2 : M2c - 1) + (hx2 ? M2c : 0)) * p.pitch + (g1 < M1c ? g1 : M1c - 1) +
                   (src ? M1c : 0);
        } else {
            valid[o] = eg2 < M2e && eg1 < M1e;
            use[o] = tid < NT && valid[o] && !(esrc + ehx2 == 0 && !e.last);
            idx = (int64_t)(eg2 + (ehx2 ? M2e : 0)) * p.pitch + eg1 + (esrc ? M1e : 0);
            near = (int64_t)((eg2 < M2e ? eg2 : M2e - 1) + (ehx2 ? M2e : 0)) * p.pitch +
                   (eg1 < M1e ? eg1 : M1e - 1) + (esrc ? M1e : 0);
        }
        idxs[o] = idx;
        // (plain mode: element 0 of the input, which this launch reads anyway)
        const int64_t ci = prox ? ch * p.plane + near : 0;
        const T u = (prox ? lv.zc : a.in)[ci], v = (prox ? lv.zp : a.in)[ci];
        zcr[o] = use[o] ? u : T(0);
        zpr[o] = use[o] ? v : T(0);
        const T w = (prox ? (p.wmap ? p.wmap : lv.zc) : a.in)[ci];  // ci indexes the Mallat plane or is 0
        wr[o] = use[o] && p.wmap ? w : T(0);
    }

    // level D input region: rows and columns 2 c0 - 20 .. 2 c0 + 61 (periodic);
    // lane = column (and column 64 + lane for the first 18 lanes), wave = rows
    constexpr int NW = NTS / 64, RPW = (BR + NW - 1) / NW;
    const int lane = tid & 63, wv = tid >> 6;
    const bool l2 = lane < BR - 64;
    const int qa = wrap(2 * c01 - 20 + lane, M1), qb = wrap(2 * c01 - 20 + 64 + (l2 ? lane : 0), M1);
    T va[RPW], vb[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        int r = wv + i * NW;
        r = r < BR ? r : BR - 1;  // past the end: an in-range duplicate, unused
        const T *rowp = in + (int64_t)wrap(2 * c02 - 20 + r, M2) * a.in_pitch;
        va[i] = rowp[qa];
        vb[i] = rowp[qb];
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int r = wv + i * NW;
        if (r < BR) {
            sIn[r][lane] = va[i];
            if (l2) sIn[r][64 + lane] = vb[i];
        }
    }
    __syncthreads();
    // along x1: level D's tile (rows 10..61, both filters, as analysis_body)
    // and the low-pass of the approximation region (all 82 rows, 36 columns)
    for (int t = tid; t < AR * (TC / 4) + BR * (LR / 4); t += NTS) {
        if (t < AR * (TC / 4)) {
            const int blk = t / AR, r = t - blk * AR;
            T x[28];
#pragma unroll
            for (int j = 0; j < 28; ++j) x[j] = sIn[10 + r][10 + 8 * blk + j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T lo = T(0), hi = T(0);
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    lo = fma(a.f.h[m], x[2 * q + m + 10], lo);
                    hi = fma(a.f.g[m], x[2 * q + m], hi);
                }
                sRow[0][r][4 * blk + q] = lo;
                sRow[1][r][4 * blk + q] = hi;
            }
        } else {
            const int t2 = t - AR * (TC / 4), blk = t2 / BR, r = t2 - blk * BR;
            T x[18];
#pragma unroll
            for (int j = 0; j < 18; ++j) x[j] = sIn[r][8 * blk + j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T lo = T(0);
#pragma unroll
                for (int m = 0; m < 12; ++m) lo = fma(a.f.h[m], x[2 * q + m], lo);
                sLo[r][4 * blk + q] = lo;
            }
        }
    }
    __syncthreads();
    // along x2: level D's tile into registers; the approximation region into sLL
    T res[4] = {T(0), T(0), T(0), T(0)};
    if (tid < NT) {
        T x[24];
#pragma unroll
        for (int j = 0; j < 24; ++j) x[j] = sRow[src][4 * rblk + j][l1];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            T lo = T(0), hi = T(0);
#pragma unroll
            for (int m = 0; m < 12; ++m) {
                lo = fma(a.f.h[m], x[2 * q + m + 10], lo);
                hi = fma(a.f.g[m], x[2 * q + m], hi);
            }
            res[2 * q + 0] = lo;
            res[2 * q + 1] = hi;
        }
    }
    constexpr int B0 = NTS > NT ? NT : 0;  // first thread of the region's x2 pass
    for (int t = tid - B0; t >= 0 && t < LR * (LR / 4); t += NTS - B0) {
        const int blk = t / LR, c = t - blk * LR;
        T x[18];
#pragma unroll
        for (int j = 0; j < 18; ++j) x[j] = sLo[8 * blk + j][c];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T lo = T(0);
#pragma unroll
            for (int m = 0; m < 12; ++m) lo = fma(a.f.h[m], x[2 * q + m], lo);
            sLL[4 * blk + q][c] = lo;
        }
    }
    __syncthreads();
    // level E along x1: 36 rows x 8 columns of both filters
    if (tid < LR * (TE / 4)) {
        const int blk = tid / LR, r = tid - blk * LR;
        T x[28];
#pragma unroll
        for (int j = 0; j < 28; ++j) x[j] = sLL[r][8 * blk + j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T lo = T(0), hi = T(0);
#pragma unroll
            for (int m = 0; m < 12; ++m) {
                lo = fma(a.f.h[m], x[2 * q + m + 10], lo);
                hi = fma(a.f.g[m], x[2 * q + m], hi);
            }
            sRowE[0][r][4 * blk + q] = lo;
            sRowE[1][r][4 * blk + q] = hi;
        }
    }
    __syncthreads();
    // level E along x2: one output per thread
    T reso = T(0);
    if (tid < NT) {
        T x[12];
        const int r0 = 2 * er + (ehx2 ? 0 : 10);
#pragma unroll
        for (int j = 0; j < 12; ++j) x[j] = sRowE[esrc][r0 + j][ec];
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < 12; ++m) acc = fma(ehx2 ? a.f.g[m] : a.f.h[m], x[m], acc);
        reso = acc;
    }

    // epilogue: level D's details, then level E's output (approximation to
    // e.apx_out unless it is the last level)
    double st[2] = {0.0, 0.0};
    bool bad = false;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        if (tid >= NT || !valid[o]) continue;
        const int b = o < 4 ? src + 2 * (o & 1) : esrc + 2 * ehx2;
        const T val = o < 4 ? res[2 * (o >> 1) + (o & 1)] : reso;
        if (o < 4 && b == 0) continue;
        if (o == 4 && b == 0 && !e.last) {
            e.apx_out[ch * e.apx_plane + (int64_t)eg2 * M1e + eg1] = val;
            continue;
        }
        if (!prox) {
            lv.zn[ch * p.plane + idxs[o]] = val;
            continue;
        }
        const int bd = o < 4 ? a.band_detail : e.band_detail;
        const T wband = b == 0 ? uniform(p.wlev[0]) : uniform(p.wlev[bd]);
        const T w = p.wmap ? wr[o] : wband;
        const T y = momentum(zcr[o], zpr[o], lv.beta);
        const T z = prox1(y, val, p.tau, w, st, bad);
        lv.zn[ch * p.plane + idxs[o]] = z;
        if (p.zsave) p.zsave[ch * p.plane + idxs[o]] = z;
    }
    if (prox) {
        if (lv.slots) block_slot_add<2, NTS>(st, lv.slots + PD_NSLOT);
        if (bad) atomicOr(p.flag, 1);
    }
}

// ===========================================================================
// Coarse levels lc..L in one workgroup per channel (per image when joint):
// everything stays in LDS.  Analysis of the level lc-1 approximation (m2 x
// m1), gradient step + prox + momentum on the coarse block of the Mallat
// plane, then synthesis of the next iteration's y back to a level lc-1
// approximation.  Same formulas as the fine kernels, periodic indices taken
// modulo the (small) band sizes.  All global loads are issued up front.
// The workgroup also finalises the iteration's statistics (it runs after
// every other kernel of the iteration).
// ===========================================================================
constexpr int NTC = 1024;
static_assert(NTC / 16 >= PD_TAIL_MAX, "tail_apply: 16 threads per output");
constexpr int CPT = 4;  // block elements per thread (64 x 64 / 1024)

// LDS geometry of the coarse kernel for blocks up to CM x CM.  The filter
// passes read periodic neighbours from halo copies written together with each
// value, so their inner loops use fixed offsets and no index wrapping.  Each
// pass computes two neighbouring outputs per task; the second of a pair that
// falls outside an odd-sized band is computed from in-bounds values and dropped.
//   A  the Mallat block (home of the coefficients), pitch PA
//   C  analysis input rows, wrapped columns HA to the left and HA+2 to the
//      right (pitch PC); later the synthesis rows with HS wrapped columns
//      before the low band and HS+1 after the high band (E, pitch PE)
//   B  analysis row-pass output with HA wrapped rows above and HA+2 below
//      (pitch PB); later the synthesis inputs D[lev]: the level's Mallat block
//      with HS wrapped rows above its low band and HS+1 below its high band
// The odd pitches PC and PE keep lane-per-row accesses free of bank conflicts.
template <typename T>
struct CGeom {
    static constexpr int CM = sizeof(T) == 4 ? 64 : 32;
    static constexpr int HA = 10, HS = 5;
    static constexpr int PA = CM + 1, PB = CM + 1;
    static constexpr int PC = CM + 2 * HA + 3, PE = CM + 2 * HS + 3;
    static constexpr int DR = 2 * HS + 1;  // halo rows of one D level
};

// Index split e -> (e / w, e % w) with a shift when w is a power of two.
__device__ __forceinline__ void split(int e, int w, int &q, int &r)
{
    if ((w & (w - 1)) == 0) {
        const int sh = __builtin_ctz(w);
        q = e >> sh;
        r = e & (w - 1);
    } else {
        q = e / w;
        r = e - q * w;
    }
}

// f(p) for every p = i + t n (t integer) with lo <= p < hi, given lo <= i < hi.
template <typename F>
__device__ __forceinline__ void copies(int i, int n, int lo, int hi, F &&f)
{
    for (int p = i - n; p >= lo; p -= n) f(p);
    f(i);
    for (int p = i + n; p < hi; p += n) f(p);
}

// First row of D[lev] (level block M2 = m2 >> lev rows).
template <typename T>
__device__ __forceinline__ int drow_base(int m2, int lev)
{
    int b = 0;
    for (int j = 0; j < lev; ++j) b += (m2 >> j) + CGeom<T>::DR;
    return b;
}

// Writes block value v at (r, c) of D[lev] (level block M2 rows, bands Mc2 = M2/2).
template <typename T>
__device__ __forceinline__ void put_d(T *D, int M2, int r, int c, T v)
{
    using G = CGeom<T>;
    const int Mc2 = M2 >> 1;
    if (r < Mc2)
        copies(r + G::HS, Mc2, 0, Mc2 + G::HS, [&](int p) { D[p * G::PB + c] = v; });
    else
        copies(r + G::HS, Mc2, Mc2 + G::HS, M2 + G::DR, [&](int p) { D[p * G::PB + c] = v; });
}

// One analysis level (Section 2.1 filters, rows then columns): the M1 x M2
// approximation in C -> detail bands in A; the approximation band goes to C
// (next level, wrapped columns) or, if `last`, to A.
template <typename T>
__device__ __forceinline__ void ana_level(T *A, T *B, T *C, int M1, int M2, const Filt<T> &f, bool last)
{
    using G = CGeom<T>;
    const int h1 = M1 / 2, h2 = M2 / 2;
    const int q1 = (h1 + 1) / 2, q2 = (h2 + 1) / 2;  // output pairs per row / column
    for (int e = threadIdx.x; e < M2 * q1; e += NTC) {  // along x1; lane = row
        int r, j;
        split(e, M2, j, r);
        const int l = 2 * j;
        const T *row = C + r * G::PC + 2 * l;  // row[k] = input column 2l+k-10
        T x[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) x[k] = row[k];
        T lo0 = T(0), hi0 = T(0), lo1 = T(0), hi1 = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            lo0 = fma(f.h[k], x[k + 10], lo0);
            hi0 = fma(f.g[k], x[k], hi0);
            lo1 = fma(f.h[k], x[k + 12], lo1);
            hi1 = fma(f.g[k], x[k + 2], hi1);
        }
        const bool two = l + 1 < h1;
        copies(r + G::HA, M2, 0, M2 + 2 * G::HA + 2, [&](int p) {
            T *br = B + p * G::PB;
            br[l] = lo0;
            br[h1 + l] = hi0;
            if (two) {
                br[l + 1] = lo1;
                br[h1 + l + 1] = hi1;
            }
        });
    }
    __syncthreads();
    for (int e = threadIdx.x; e < q2 * M1; e += NTC) {  // along x2; lane = column
        int j, c;
        split(e, M1, j, c);
        const int l = 2 * j;
        const T *col = B + 2 * l * G::PB + c;  // col[k PB] = row 2l+k-10
        T x[24];
#pragma unroll
        for (int k = 0; k < 24; ++k) x[k] = col[k * G::PB];
        T lo0 = T(0), hi0 = T(0), lo1 = T(0), hi1 = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            lo0 = fma(f.h[k], x[k + 10], lo0);
            hi0 = fma(f.g[k], x[k], hi0);
            lo1 = fma(f.h[k], x[k + 12], lo1);
            hi1 = fma(f.g[k], x[k + 2], hi1);
        }
        const bool two = l + 1 < h2;
        if (c < h1 && !last) {
            copies(c + G::HA, h1, 0, h1 + 2 * G::HA + 2, [&](int p) {
                C[l * G::PC + p] = lo0;
                if (two) C[(l + 1) * G::PC + p] = lo1;
            });
        } else {
            A[l * G::PA + c] = lo0;
            if (two) A[(l + 1) * G::PA + c] = lo1;
        }
        A[(h2 + l) * G::PA + c] = hi0;
        if (two) A[(h2 + l + 1) * G::PA + c] = hi1;
    }
    __syncthreads();
}

// Two synthesis outputs (parities 0, 1) of one position pp from lo[j] =
// low band at pp-5+j and hi[j] = high band at pp+j (j = 0..5).
template <typename T>
__device__ __forceinline__ void syn_pair(const Filt<T> &f, const T *lo, const T *hi, T &o0, T &o1)
{
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        a0 = fma(f.h[10 - 2 * j], lo[j], a0);
        a0 = fma(f.g[10 - 2 * j], hi[j], a0);
        a1 = fma(f.h[11 - 2 * j], lo[j], a1);
        a1 = fma(f.g[11 - 2 * j], hi[j], a1);
    }
    o0 = a0;
    o1 = a1;
}

// One synthesis level: the M1 x M2 Mallat block in D (bands M1/2 x M2/2) ->
// the M1 x M2 approximation, written to D of the next finer level (its
// approximation band, that level has M2n = 2 M2 rows) or, for the finest
// level (Dn == nullptr), to A.
template <typename T>
__device__ __forceinline__ void syn_level(const T *D, T *E, T *Dn, int M2n, T *A, int M1, int M2, const Filt<T> &f)
{
    using G = CGeom<T>;
    const int M1c = M1 / 2, M2c = M2 / 2;
    const int q2 = (M2c + 1) / 2, q1 = (M1c + 1) / 2;
    for (int e = threadIdx.x; e < q2 * M1; e += NTC) {  // along x2; lane = column
        int j0, c;
        split(e, M1, j0, c);
        const int pp = 2 * j0;
        const T *lo_p = D + pp * G::PB + c;                  // rows pp-5 .. pp+1 of the low band
        const T *hi_p = D + (M2c + G::HS + pp) * G::PB + c;  // rows pp .. pp+6 of the high band
        T lo[7], hi[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            lo[j] = lo_p[j * G::PB];
            hi[j] = hi_p[j * G::PB];
        }
        T o[4];
        syn_pair<T>(f, lo, hi, o[0], o[1]);
        syn_pair<T>(f, lo + 1, hi + 1, o[2], o[3]);
        const int nout = pp + 1 < M2c ? 4 : 2;
        const bool low = c < M1c;
        copies(c + G::HS, M1c, low ? 0 : M1c + G::HS, low ? M1c + G::HS : M1 + G::DR, [&](int p) {
            for (int q = 0; q < 4; ++q)
                if (q < nout) E[(2 * pp + q) * G::PE + p] = o[q];
        });
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M2 * q1; e += NTC) {  // along x1; lane = row
        int n, j0;
        split(e, M2, j0, n);
        const int pp = 2 * j0;
        const T *row = E + n * G::PE;
        T lo[7], hi[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            lo[j] = row[pp + j];
            hi[j] = row[M1c + G::HS + pp + j];
        }
        T o[4];
        syn_pair<T>(f, lo, hi, o[0], o[1]);
        syn_pair<T>(f, lo + 1, hi + 1, o[2], o[3]);
        const int nout = pp + 1 < M1c ? 4 : 2;
        if (Dn) {
            // approximation band of the finer level: low band rows, wrapped above
            copies(n + G::HS, M2, 0, M2 + G::HS, [&](int p) {
                for (int q = 0; q < 4; ++q)
                    if (q < nout) Dn[p * G::PB + 2 * pp + q] = o[q];
            });
        } else {
            for (int q = 0; q < 4; ++q)
                if (q < nout) A[n * G::PA + 2 * pp + q] = o[q];
        }
    }
    __syncthreads();
    (void)M2n;
}

// The tail: out = Mat in over the tM2 x tM1 approximation at the top-left of A
// (tn <= PD_TAIL_MAX values), 16 threads per output, fixed summation order.
template <typename T>
__device__ void tail_apply(T *A, int tM1, int tM2, const T *Mat, T *Dout = nullptr, int DM2 = 0)
{
    using G = CGeom<T>;
    const int tn = tM1 * tM2;
    const int i = threadIdx.x >> 4, q = threadIdx.x & 15;
    T acc = T(0);
    if (i < tn) {
        const T *row = Mat + i * tn;
        for (int j = q; j < tn; j += 16) {
            int r, c;
            split(j, tM1, r, c);
            acc = fma(row[j], A[r * G::PA + c], acc);
        }
    }
    acc = dpp_row_sum(acc);  // the 16 threads of an output form one DPP row
    __syncthreads();         // every read of A is done
    if (i < tn && q == 0) {
        int r, c;
        split(i, tM1, r, c);
        if (Dout)  // approximation band of the coarsest pass-by-pass synthesis level
            put_d<T>(Dout, DM2, r, c, acc);
        else
            A[r * G::PA + c] = acc;
    }
    __syncthreads();
}

// Analysis of the block in A: kw levels pass by pass, then the tail as one matrix.
template <typename T>
__device__ void coarse_analysis(T *A, T *B, T *C, int m1, int m2, int nlev, const Filt<T> &f, int kw, int tM1,
                                int tM2, const T *Mat, bool in_c)
{
    using G = CGeom<T>;
    if (kw > 0 && !in_c) {  // (in_c: the input was staged in C at load time)
        for (int e = threadIdx.x; e < m1 * m2; e += NTC) {
            int r, c;
            split(e, m1, r, c);
            const T v = A[r * G::PA + c];
            copies(c + G::HA, m1, 0, m1 + 2 * G::HA + 2, [&](int p) { C[r * G::PC + p] = v; });
        }
        __syncthreads();
    }
    for (int lev = 0; lev < kw; ++lev) ana_level<T>(A, B, C, m1 >> lev, m2 >> lev, f, lev == kw - 1);
    if (kw < nlev) tail_apply<T>(A, tM1, tM2, Mat);
}

// Synthesis of the block in A: the tail (transposed matrix), then kw levels
// coarse to fine; the result replaces the block in A.
template <typename T>
__device__ void coarse_synthesis(T *A, T *D, T *E, int m1, int m2, int nlev, const Filt<T> &f, int kw, int tM1,
                                 int tM2, const T *MatT, bool routed)
{
    using G = CGeom<T>;
    if (routed) {  // the details are already in D: only the tail remains, straight into D
        if (kw < nlev) tail_apply<T>(A, tM1, tM2, MatT, D + drow_base<T>(m2, kw - 1) * G::PB, m2 >> (kw - 1));
        goto levels;
    }
    if (kw < nlev) tail_apply<T>(A, tM1, tM2, MatT);
    if (kw == 0) return;
    // every coefficient of the block goes to the input of the level that reads it
    for (int e = threadIdx.x; e < m1 * m2; e += NTC) {
        int r, c;
        split(e, m1, r, c);
        int lev = kw - 1;
        for (int j = 0; j < kw - 1; ++j)
            if (r >= (m2 >> (j + 1)) || c >= (m1 >> (j + 1))) {
                lev = j;
                break;
            }
        put_d<T>(D + drow_base<T>(m2, lev) * G::PB, m2 >> lev, r, c, A[r * G::PA + c]);
    }
    __syncthreads();
levels:
    for (int lev = kw - 1; lev >= 0; --lev) {
        const T *Dl = D + drow_base<T>(m2, lev) * G::PB;
        T *Dn = lev > 0 ? D + drow_base<T>(m2, lev - 1) * G::PB : nullptr;
        syn_level<T>(Dl, E, Dn, lev > 0 ? (m2 >> (lev - 1)) : 0, A, m1 >> lev, m2 >> lev, f);
    }
}

// LDS layout of the coarse kernel (elements): A per channel, C/E, B/D, tail matrices.
template <typename T>
struct CLayout {
    int a, c, b, mat, total;
    __host__ __device__ CLayout(int m1, int m2, int nch)
    {
        using G = CGeom<T>;
        a = 0;
        c = a + nch * m2 * G::PA;
        b = c + m2 * G::PC;
        int drows = 0;  // levels done pass by pass hold more than PD_TAIL_MAX values
        for (int j = 0; (m1 >> j) * (m2 >> j) > PD_TAIL_MAX; ++j) drows += (m2 >> j) + G::DR;
        const int brows = m2 + 2 * G::HA + 2;
        mat = b + (drows > brows ? drows : brows) * G::PB + 8;  // + 8: reads past a dropped pair
        total = mat + 2 * PD_TAIL_MAX * PD_TAIL_MAX;
    }
};

template <typename T>
__device__ __forceinline__ T beta_at(int i);  // (below, with the reverse kernels)

// NCH: channels handled by the workgroup (the joint colour prox couples them);
// JOINT: the prox is the joint (group) one -- a compile-time choice, so the
// scalar kernel carries no code of the other.  SM, SKW, STM, SNL, SOPS: when
// nonzero, the block side (square), the number of pass-by-pass levels, the
// tail side, the number of levels and the operations as compile-time
// constants (the arguments then hold the same values): the common geometry
// gets its index arithmetic folded at compile time.
template <typename T, int NCH, bool JOINT, int SM = 0, int SKW = 0, int STM = 0, int SNL = 0, int SOPS = 0>
__device__ __forceinline__ void coarse_body(const CoarseArgs<T> &a, const Live<T> &lv, int bz)
{
    using G = CGeom<T>;
    extern __shared__ unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    const ProxArgs<T> &p = a.p;
    const int m1 = SM ? SM : a.m1, m2 = SM ? SM : a.m2;
    const int kw = SKW ? SKW : a.kw;
    const int tM1 = STM ? STM : a.tM1, tM2 = STM ? STM : a.tM2;
    const int nlev = SNL ? SNL : a.nlev, ops = SOPS ? SOPS : a.ops;
    const int ch0 = NCH > 1 ? 0 : bz;
    const CLayout<T> L(m1, m2, NCH);
    T *Cb = lds + L.c;
    T *B = lds + L.b;
    T *Mat = lds + L.mat;  // [2][tn][tn] tail matrices
    const int tn = tM1 * tM2;
    const int cnt = m1 * m2;  // <= CPT * NTC
    const int tid = threadIdx.x;
    const bool ana = (ops & COARSE_ANA) != 0, prox = (ops & COARSE_PROX) != 0;
    const bool revcm = NCH == 1 && !JOINT && (ops & COARSE_REVCM) != 0;
    const bool need_z = !ana || prox || revcm;
    const bool routed = NCH == 1 && !JOINT && ana && (prox || revcm) && (ops & COARSE_SYN) && kw > 0;
    auto home = [&](int cc) { return lds + L.a + cc * m2 * G::PA; };

    // 1. every global load at once (clamped indices, no data-dependent branch):
    //    analysis input or y's state, prox state and weights, tail matrices
    int rr[CPT], cr[CPT];
    int64_t gi[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        const int e = tid + k * NTC;
        split(e < cnt ? e : 0, m1, rr[k], cr[k]);
        gi[k] = (int64_t)rr[k] * p.pitch + cr[k];
    }
    // an unused source is replaced by element 0 of a buffer this launch reads anyway
    const T *any = ana ? a.apx_in : lv.zc;
    auto ld = [&](const T *src, bool use, int64_t i) {
        const T x = (use ? src : any)[use ? i : 0];
        return use ? x : T(0);
    };
    T v[NCH][CPT], zcr[NCH][CPT], zpr[NCH][CPT], wr[CPT];
#pragma unroll
    for (int cc = 0; cc < NCH; ++cc)
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int e = tid + k * NTC;
            const int64_t ch = ch0 + cc;
            v[cc][k] = ld(a.apx_in, ana, ch * a.apx_in_plane + (e < cnt ? e : 0));
            zcr[cc][k] = ld(lv.zc, need_z, ch * p.plane + gi[k]);
            zpr[cc][k] = ld(lv.zp, need_z, ch * p.plane + gi[k]);
        }
    const bool use_w = prox && p.wmap;
#pragma unroll
    for (int k = 0; k < CPT; ++k) wr[k] = ld(p.wmap, use_w, (int64_t)ch0 * p.plane + gi[k]);
    __shared__ T wtab[PD_MAXL + 1];  // band weights, read per coefficient by the prox
    if (tid <= PD_MAXL) {  // selects between scalar argument values: no per-lane argument load
        T wv = uniform(p.wlev[0]);
#pragma unroll
        for (int k = 1; k <= PD_MAXL; ++k) wv = tid == k ? uniform(p.wlev[k]) : wv;
        wtab[tid] = wv;
    }
    constexpr int MPT = 2 * PD_TAIL_MAX * PD_TAIL_MAX / NTC;
    static_assert(MPT * NTC == 2 * PD_TAIL_MAX * PD_TAIL_MAX, "tail matrix slots: every thread stores MPT");
    T mv[MPT];
    const int nm = a.tail ? 2 * tn * tn : 0;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int e = tid + k * NTC;
        mv[k] = ld(a.tail, nm > 0, e < nm ? e : 0);
    }
#pragma unroll
    for (int k = 0; k < MPT; ++k)  // unconditional (slots past 2 tn^2 are unused), so that no
        Mat[tid + k * NTC] = mv[k];  // load is deferred into a branch behind a full wait
    // one channel with pass-by-pass levels: the analysis input goes straight
    // into C with its wrapped columns
    const bool in_c = NCH == 1 && ana && kw > 0;
#pragma unroll
    for (int cc = 0; cc < NCH; ++cc)
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (tid + k * NTC < cnt) {
                if (in_c) {
                    const T x = v[cc][k];
                    copies(cr[k] + G::HA, m1, 0, m1 + 2 * G::HA + 2, [&](int q) { Cb[rr[k] * G::PC + q] = x; });
                } else {
                    home(cc)[rr[k] * G::PA + cr[k]] =
                        ana ? v[cc][k] : momentum(zcr[cc][k], zpr[cc][k], lv.beta);
                }
            }
    __syncthreads();

    if (ana) {
#pragma unroll
        for (int cc = 0; cc < NCH; ++cc)
            coarse_analysis<T>(home(cc), B, Cb, m1, m2, nlev, a.f, kw, tM1, tM2, Mat, in_c);
        if constexpr (NCH == 1 && !JOINT) {
            if (revcm) {
                // reverse sweep: combine of iteration i, mask of iteration i-1
                // (the element-wise kernels' formulas), the new vbar routed to
                // the synthesis like y(i+1) in the prox branch
                T b = a.rv_b;
                int first = a.rv_first;
                if (a.rv_di.it_dev) {
                    const int i = *a.rv_di.it_dev + a.rv_di.it_off;
                    b = beta_at<T>(i);
                    first = i == 1;
                }
                T zbm[CPT], wb[CPT];
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const int64_t gidx = (int64_t)ch0 * p.plane + gi[k];
                    zbm[k] = a.rv_zbarm[gidx];
                    wb[k] = (a.rv_wbar ? a.rv_wbar : a.rv_zbarm)[gidx];
                }
                T *A = home(0);
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (tid + k * NTC >= cnt) continue;
                    const int r = rr[k], c = cr[k];
                    const int li = r * G::PA + c;
                    const int64_t gidx = (int64_t)ch0 * p.plane + gi[k];
                    const T yb = fma(-p.tau, A[li], zcr[0][k]);
                    T zb;
                    if (first) {
                        zb = yb + zbm[k];
                    } else {
                        zb = fma(T(1) + b, yb, zbm[k]);
                        a.rv_zbarm[gidx] = -b * yb;
                    }
                    a.rv_zbar[gidx] = zb;
                    const T zv = zpr[0][k];
                    const bool act = zv != T(0);
                    const T vn = act ? zb : T(0);
                    a.rv_vbar[gidx] = vn;
                    if (a.rv_wbar && act) {
                        const T t = p.tau * zb;
                        a.rv_wbar[gidx] = wb[k] - (zv > T(0) ? t : -t);
                    }
                    if (!routed || (kw < nlev && r < tM2 && c < tM1)) {
                        A[li] = vn;
                    } else {
                        int lev = kw - 1;
                        for (int j = 0; j < kw - 1; ++j)
                            if (r >= (m2 >> (j + 1)) || c >= (m1 >> (j + 1))) {
                                lev = j;
                                break;
                            }
                        put_d<T>(B + drow_base<T>(m2, lev) * G::PB, m2 >> lev, r, c, vn);
                    }
                }
                __syncthreads();
            }
        }
        if (!prox && !revcm) {  // plain forward transform
#pragma unroll
            for (int cc = 0; cc < NCH; ++cc)
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    if (tid + k * NTC < cnt)
                        lv.zn[(int64_t)(ch0 + cc) * p.plane + gi[k]] = home(cc)[rr[k] * G::PA + cr[k]];
            return;
        }
        // 2. gradient step + prox + momentum on the coarse block; with one
        //    channel and a synthesis to follow, y(i+1) is routed to where the
        //    synthesis reads it
        if (prox) {
        double st[2] = {0.0, 0.0};
        bool bad = false;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if (tid + k * NTC >= cnt) continue;
            const int r = rr[k], c = cr[k];
            // band weight: the levels whose approximation region holds (r, c) are
            // counted (branch-free); all of them -> the approximation band (k = 0),
            // else the detail band of the first level that does not
            int inside = 0;
            for (int lev = 0; lev < nlev; ++lev)  // uniform trip count
                inside += (r < (m2 >> (lev + 1))) & (c < (m1 >> (lev + 1)));
            const int band = inside == nlev ? 0 : a.band_top - inside;
            const T wband = wtab[band];
            const int li = r * G::PA + c;
            if (!JOINT) {
                T *A = home(0);
                T w = p.wmap ? wr[k] : wband;
                T y = momentum(zcr[0][k], zpr[0][k], lv.beta);
                T z = prox1(y, A[li], p.tau, w, st, bad);
                lv.zn[(int64_t)ch0 * p.plane + gi[k]] = z;
                if (p.zsave) p.zsave[(int64_t)ch0 * p.plane + gi[k]] = z;
                const T yn = momentum(z, zcr[0][k], lv.beta_next);
                if (!routed || (kw < nlev && r < tM2 && c < tM1)) {
                    A[li] = yn;  // the tail's input (or the whole block)
                } else {  // straight into the synthesis input of the level that reads it
                    int lev = kw - 1;
                    for (int j = 0; j < kw - 1; ++j)
                        if (r >= (m2 >> (j + 1)) || c >= (m1 >> (j + 1))) {
                            lev = j;
                            break;
                        }
                    put_d<T>(B + drow_base<T>(m2, lev) * G::PB, m2 >> lev, r, c, yn);
                }
            } else {
                T yv[NCH], vv[NCH];
                T nv = T(0);
                double ny = 0.0;
#pragma unroll
                for (int cc = 0; cc < NCH; ++cc) {
                    yv[cc] = momentum(zcr[cc][k], zpr[cc][k], lv.beta);
                    vv[cc] = grad_step(yv[cc], home(cc)[li], p.tau);
                    nv = fma(vv[cc], vv[cc], nv);
                    ny += (double)yv[cc] * (double)yv[cc];
                }
                T w = wband;
                T nrm = sqrt(nv);
                T sc = nrm > T(0) ? T(1) - p.tau * w / nrm : T(0);
                sc = sc > T(0) ? sc : T(0);
                bad |= !isfinite(nrm);
                st[0] += (double)w * sqrt(ny);
#pragma unroll
                for (int cc = 0; cc < NCH; ++cc) {
                    T z = mul_rn(vv[cc], sc);
                    lv.zn[(int64_t)cc * p.plane + gi[k]] = z;
                    if (p.zsave) p.zsave[(int64_t)cc * p.plane + gi[k]] = z;
                    st[1] += ((double)z - (double)yv[cc]) * ((double)z - (double)yv[cc]);
                    home(cc)[li] = momentum(z, zcr[cc][k], lv.beta_next);
                }
            }
        }
        if (bad) atomicOr(p.flag, 1);
        if (lv.slots) block_slot_add<2, NTC>(st, lv.slots + PD_NSLOT);  // contains a barrier
        else __syncthreads();
        }
    }
    if (!(ops & COARSE_SYN)) return;
    // 3. synthesis of the block back to the level lc-1 approximation
#pragma unroll
    for (int cc = 0; cc < NCH; ++cc) {
        T *A = home(cc);
        coarse_synthesis<T>(A, B, Cb, m1, m2, nlev, a.f, kw, tM1, tM2, Mat + tn * tn, routed);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int e = tid + k * NTC;
            if (e < cnt) a.apx_out[(int64_t)(ch0 + cc) * a.apx_out_plane + e] = A[rr[k] * G::PA + cr[k]];
        }
    }
}

// Statistics finaliser: workgroup (j, img) sums ring entry (it0+j) % PD_RING
// of image img into stats[it0+j][0..2] and zeroes the entry.
__device__ void finalize_entry(double *slots, double *stats)
{
    __shared__ double red[3][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v[3] = {0.0, 0.0, 0.0};
    for (int e = threadIdx.x; e < PD_NSLOT; e += 256) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            v[q] += slots[q * PD_NSLOT + e];
            slots[q * PD_NSLOT + e] = 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double a = v[q];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) red[q][wv] = a;
    }
    __syncthreads();
    if (threadIdx.x < 3) stats[threadIdx.x] += red[threadIdx.x][0] + red[threadIdx.x][1] +
                                               red[threadIdx.x][2] + red[threadIdx.x][3];
}

__global__ __launch_bounds__(256) void k_stats_finalize(double *ring, double *stats, int it0)
{
    const int it = it0 + blockIdx.x;
    finalize_entry(ring + (size_t)(it % PD_RING) * 3 * PD_NSLOT, stats + 3 * (size_t)it);
}

__global__ __launch_bounds__(256) void k_stats_finalize_dev(double *ring, double *stats, const int *it_dev, int sub)
{
    const int it = *it_dev - sub + blockIdx.x;
    finalize_entry(ring + (size_t)(it % PD_RING) * 3 * PD_NSLOT, stats + 3 * (size_t)it);
}

__global__ void k_set_int(int *dst, int v)
{
    if (threadIdx.x == 0) dst[0] = v;
}

__global__ __launch_bounds__(256) void k_stats_finalize_b(double *const *__restrict__ ring,
                                                           double *const *__restrict__ stats, int it0,
                                                           const int *it_dev)
{
    const int it = (it_dev ? *it_dev : 0) + it0 + blockIdx.x, img = blockIdx.y;
    finalize_entry(ring[img] + (size_t)(it % PD_RING) * 3 * PD_NSLOT, stats[img] + 3 * (size_t)it);
}

template <typename T>
__global__ void k_fill(T *dst, T v, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = v;
}

// ===========================================================================
// Blur (Section 1, eq. 1.1; Operator 1 of Section 4.1): with the profile
// k_{y2} of source row y2,
//   t(x1,y2)  = sum_d k_{y2}[d] x(x1-d, y2)             (rows, own profile)
//   Hx(x1,x2) = sum_d k_{x2-d}[d] t(x1, x2-d)           (columns, source profile)
//   r = Hx - f0
//   u(x1,y2)  = sum_d k_{y2}[d] r(x1, y2+d)             (H^T: columns)
//   s(y1,y2)  = sum_d k_{y2}[d] u(y1+d, y2)             (H^T: rows)
// A workgroup produces a BT2-row x 46-column tile of s, so the column passes
// work on exactly 64 columns: one wave64 per block of rows with lane = column,
// which makes the row profiles wave-uniform (scalar loads).  Profiles narrower
// than RM = 9 are zero-padded.
// ===========================================================================
constexpr int RM = PD_MAX_RADIUS;
constexpr int BW = 64;                 // columns of t, r, u
constexpr int BT1 = BW - 2 * RM;       // 46 output columns
constexpr int BX1 = BT1 + 4 * RM;      // 82 x columns
constexpr int XP = 84;                 // LDS pitch of x (multiple of 4)
constexpr int TP = 68;                 // LDS pitch of t, r, u (multiple of 4)
// Blur workgroup: 1024 threads for the FP32 32-row tile (four waves per SIMD,
// every pass's tasks in one round), else 512 (two waves per SIMD hide the LDS
// latency; 1024 would spill).  The same outputs either way.
template <typename T, int BT2>
constexpr int blur_threads() { return sizeof(T) == 4 && BT2 == 32 ? 1024 : 512; }
static_assert(BX1 <= 128 && BX1 > 64, "blur load columns");
constexpr int UVH = 4;                 // rows per column task in the u pass

// Tile height variants (the tuned parameter; every output pixel is computed by
// the same sums in the same order whatever the variant): BT2 output rows,
// BX2 rows of x and t, BR2 rows of r, RVH rows per column task of the r pass.
template <int BT2_, int NTB>
struct BlurGeom {
    static constexpr int BT2 = BT2_;
    static constexpr int BX2 = BT2 + 4 * RM;
    static constexpr int BR2 = BT2 + 2 * RM;
    static constexpr int RVH = BT2 == 32 ? 5 : 6;  // divides BR2 (50 = 10 x 5, 66 = 11 x 6)
    static constexpr int RB_PER_WAVE = (BR2 / RVH + NTB / 64 - 1) / (NTB / 64);  // r-pass row blocks per wave
    static_assert(BR2 % RVH == 0 && BT2 % UVH == 0, "blur pass blocking");
};

template <typename T, int BT2>
struct BlurLds {
    using G = BlurGeom<BT2, blur_threads<T, BT2>()>;
    alignas(16) T sA[G::BX2 * XP];         // x, later r (BR2 x TP)
    alignas(16) T sB[G::BX2 * TP];         // t, later u (BT2 x TP)
    alignas(16) T sK[G::BX2][2 * RM + 2];  // profiles of the rows of x / t
    alignas(16) T sKT[G::BR2][2 * RM + 2]; // by output row of H: sKT[q][RM+d] = profile of source row q+RM-d at d
};

// The four passes on a staged tile (profiles zero-padded to RM).
template <typename T, int BT2, int NTB = blur_threads<T, BT2>(), typename G = BlurGeom<BT2, NTB>>
__device__ __forceinline__ void blur_body(const BlurArgs<T> &a, int bx, int by, int bz, BlurLds<T, BT2> &lds,
                                          const T (&f0pre)[G::RB_PER_WAVE][G::RVH])
{
    constexpr int BX2 = G::BX2, BR2 = G::BR2, RVH = G::RVH, RB_PER_WAVE = G::RB_PER_WAVE;
    T *__restrict__ sA = lds.sA;
    T *__restrict__ sB = lds.sB;
    T(*__restrict__ sK)[2 * RM + 2] = lds.sK;
    const int n1 = a.n1, n2 = a.n2;
    const int64_t ch = bz;
    const int o1 = bx * BT1, o2 = by * BT2;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

    // t: rows [0, BX2) (pixel row o2-2RM+r), columns [0, BW) (pixel col o1-RM+c)
    for (int t = tid; t < BX2 * (BW / 4); t += NTB) {
        int r = t / (BW / 4), blk = t - r * (BW / 4);
        T xv[4 + 2 * RM];
#pragma unroll
        for (int j = 0; j < 4 + 2 * RM; ++j)
            xv[j] = sA[r * XP + 4 * blk + j];
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int m = 0; m <= 2 * RM; ++m) {
            T k = sK[r][2 * RM - m];  // d = RM - m
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fma(k, xv[q + m], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) sB[r * TP + 4 * blk + q] = acc[q];
    }
    // the r pass's taps gathered by output row (contiguous in d, like the u pass)
    for (int e = tid; e < BR2 * (2 * RM + 1); e += NTB) {
        const int q = e / (2 * RM + 1), i = e - q * (2 * RM + 1);  // i = RM + d
        lds.sKT[q][i] = sK[q + 2 * RM - i][i];
    }
    __syncthreads();

    // r: rows [0, BR2) (pixel row o2-RM+r), lane = column.  Output row q =
    // r0+k gathers t rows q+RM-d (tile index k+2RM-i with i = RM+d) with the
    // taps sKT[q][i] of those source rows.
    double st[1] = {0.0};
#pragma unroll
    for (int j = 0; j < RB_PER_WAVE; ++j) {
        const int blk = wv + j * (NTB / 64);
        if (blk >= BR2 / RVH) break;
        const int r0 = blk * RVH;
        T tv[RVH + 2 * RM];
#pragma unroll
        for (int m = 0; m < RVH + 2 * RM; ++m) tv[m] = sB[(r0 + m) * TP + lane];
        T acc[RVH];
#pragma unroll
        for (int k = 0; k < RVH; ++k) {
            const T *kt = lds.sKT[r0 + k];
            T s0 = T(0);
#pragma unroll
            for (int i = 0; i <= 2 * RM; ++i) s0 = fma(kt[i], tv[k + 2 * RM - i], s0);
            acc[k] = s0;
        }
#pragma unroll
        for (int k = 0; k < RVH; ++k) {
            T rv = acc[k] - f0pre[j][k];
            sA[(r0 + k) * TP + lane] = rv;
            const int pr = r0 + k, pc = lane;
            bool own = pr >= RM && pr < RM + BT2 && pc >= RM && pc < RM + BT1 &&
                       (o2 - RM + pr) < n2 && (o1 - RM + pc) < n1;
            if (own) {
                st[0] += 0.5 * (double)rv * (double)rv;
                if (a.racc) {  // reverse mode: accumulate rscale * H x
                    T *ra = a.racc + ch * a.plane + (int64_t)(o2 - RM + pr) * n1 + (o1 - RM + pc);
                    *ra = fma(a.rscale, rv, *ra);
                }
            }
        }
    }
    __syncthreads();

    // u: rows [0, BT2) (pixel row o2+q), lane = column; output-row profile
    for (int blk = wv; blk < BT2 / UVH; blk += NTB / 64) {
        const int q0 = blk * UVH;
        T rv[UVH + 2 * RM];
#pragma unroll
        for (int j = 0; j < UVH + 2 * RM; ++j)
            rv[j] = sA[(q0 + j) * TP + lane];
#pragma unroll
        for (int k = 0; k < UVH; ++k) {
            const T *kr = &sK[q0 + k + 2 * RM][RM];  // profile of output row o2+q0+k
            T acc = T(0);
#pragma unroll
            for (int d = -RM; d <= RM; ++d) acc = fma(kr[d], rv[k + RM + d], acc);
            sB[(q0 + k) * TP + lane] = acc;
        }
    }
    __syncthreads();

    // s: rows [0, BT2), output columns [0, BT1) (pixel col o1+c)
    T *s = a.s + ch * a.plane;
    for (int t = tid; t < BT2 * ((BT1 + 3) / 4); t += NTB) {
        int q = t / ((BT1 + 3) / 4), blk = t - q * ((BT1 + 3) / 4);
        T uv[4 + 2 * RM];
#pragma unroll
        for (int j = 0; j < 4 + 2 * RM; ++j) {
            int c = 4 * blk + j;
            uv[j] = c < BW ? sB[q * TP + c] : T(0);
        }
        T acc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int m = 0; m <= 2 * RM; ++m) {
            T k = sK[q + 2 * RM][m];  // d = m - RM
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = fma(k, uv[j + m], acc[j]);
        }
        const int gy = o2 + q;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int c = 4 * blk + j, gx = o1 + c;
            if (c < BT1 && gy < n2 && gx < n1) s[(int64_t)gy * n1 + gx] = acc[j];
        }
    }
    if (a.slots) block_slot_add<1, NTB>(st, a.slots);
}

// Stages the x tile and the row profiles in LDS (with f0 prefetched for the
// r pass), then runs the passes.
template <typename T, int BT2>
__device__ __forceinline__ void blur_tile(const BlurArgs<T> &a, int bx, int by, int bz)
{
    constexpr int NTB = blur_threads<T, BT2>();
    using G = BlurGeom<BT2, NTB>;
    constexpr int BX2 = G::BX2, BR2 = G::BR2, RVH = G::RVH, RB_PER_WAVE = G::RB_PER_WAVE;
    __shared__ BlurLds<T, BT2> lds;
    T *__restrict__ sA = lds.sA;
    T(*__restrict__ sK)[2 * RM + 2] = lds.sK;
    const int n1 = a.n1, n2 = a.n2, R = a.R, W = 2 * R + 1;
    const int o1 = bx * BT1, o2 = by * BT2;
    const T *x = a.x + (int64_t)bz * a.plane;
    const T *__restrict__ taps = a.taps;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    T f0pre[RB_PER_WAVE][RVH];
    {
        // load: lane = column (two chunks: 64 + 18), wave = rows (every 8th)
        constexpr int RPW = (BX2 + NTB / 64 - 1) / (NTB / 64);
        const int qa = wrap(o1 - 2 * RM + lane, n1);
        const bool okb = 64 + lane < BX1;
        const int qb = okb ? wrap(o1 - 2 * RM + 64 + lane, n1) : 0;
        T va[RPW], vb[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + i * (NTB / 64);  // rows past BX2 read row o2-2RM, unused
            const T *rowp = x + (int64_t)wrap(o2 - 2 * RM + (r < BX2 ? r : 0), n2) * n1;
            va[i] = rowp[qa];
            vb[i] = okb ? rowp[qb] : T(0);
        }
        constexpr int KE = BX2 * (2 * RM + 1), KPT = (KE + NTB - 1) / NTB;
        T kv[KPT];
#pragma unroll
        for (int i = 0; i < KPT; ++i) {  // all profile loads in flight together
            const int e = tid + i * NTB;
            const int r = e / (2 * RM + 1), d = e - r * (2 * RM + 1) - RM;
            const bool ok = e < KE && d >= -R && d <= R;
            const int rr = r < BX2 ? r : BX2 - 1, dd = d < -R ? -R : (d > R ? R : d);  // in-range neighbour
            const T k = taps[(int64_t)wrap(o2 - 2 * RM + rr, n2) * W + dd + R];
            kv[i] = ok ? k : T(0);
        }
        // f0 for the r pass (rows of the wave's row blocks, lane = column)
        const T *f0s = a.f0 ? a.f0 + (int64_t)bz * a.plane : x;
        const int fq1 = wrap(o1 - RM + lane, n1);
#pragma unroll
        for (int j = 0; j < RB_PER_WAVE; ++j)
#pragma unroll
            for (int k = 0; k < RVH; ++k) {
                const int rr = (wv + j * (NTB / 64)) * RVH + k;
                const T f = f0s[(int64_t)wrap(o2 - RM + (rr < BR2 ? rr : BR2 - 1), n2) * n1 + fq1];
                f0pre[j][k] = a.f0 ? f : T(0);
            }
#pragma unroll
        for (int i = 0; i < KPT; ++i) {
            const int e = tid + i * NTB;
            const int r = e / (2 * RM + 1), d = e - r * (2 * RM + 1) - RM;
            if (e < KE) sK[r][d + RM] = kv[i];
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + i * (NTB / 64);
            if (r < BX2) {
                sA[r * XP + lane] = va[i];
                if (okb) sA[r * XP + 64 + lane] = vb[i];
            }
        }
    }
    __syncthreads();
    blur_body<T, BT2>(a, bx, by, bz, lds, f0pre);
}

// H = Id: s = r = x - f0.
template <typename T>
__global__ __launch_bounds__(NT) void k_identity(BlurArgs<T> a)
{
    double st[1] = {0.0};
    const int64_t total = (int64_t)a.n1 * a.n2 * a.C;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
        T rv = a.x[e] - (a.f0 ? a.f0[e] : T(0));
        a.s[e] = rv;
        st[0] += 0.5 * (double)rv * (double)rv;
        if (a.racc) a.racc[e] = fma(a.rscale, rv, a.racc[e]);
    }
    if (a.slots) block_slot_add<1, NT>(st, a.slots);
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

// ---------------------------------------------------------------------------
// Reverse mode of the iteration (adjoint of Appendix A.1's recursion).
// With z(i) = S_{tau w}(v(i)):  vbar = zbar 1{z(i) != 0},
// wbar -= tau zbar sign(z(i)) 1{z(i) != 0}  (z != 0 exactly when |v| > tau w,
// and then sign z = sign v; the kink gets derivative 0).
template <typename T>
__global__ void k_rev_mask(const T *zbar, const T *z, T *vbar, T *wbar, T tau, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const T zv = z[e], zb = zbar[e];
        const bool act = zv != T(0);
        vbar[e] = act ? zb : T(0);
        if (wbar && act) {
            const T t = tau * zb;
            wbar[e] = wbar[e] - (zv > T(0) ? t : -t);
        }
    }
}

// Momentum of y(i) = z(i-1) + b (z(i-1) - z(i-2)): b = (i-2)/(i+1), 0 for i = 1
// (Appendix A.1), in double then rounded to T exactly as on the host.
template <typename T>
__device__ __forceinline__ T beta_at(int i)
{
    return i >= 2 ? (T)((double)(i - 2) / (double)(i + 1)) : T(0);
}

// ybar = vbar - tau gbar; with b = b_{i-1}:  zbar <- zbarm + (1+b) ybar,
// zbarm <- -b ybar  (i >= 2); for i = 1 zbar <- ybar + zbarm (the init's adjoint).
template <typename T>
__global__ void k_rev_combine(const T *vbar, const T *gbar, T *zbar, T *zbarm, T tau, T b, int first, int64_t n,
                              DevIter di)
{
    if (di.it_dev) {  // iteration i from device memory (graph replay): b = b_{i-1}, first = (i == 1)
        const int i = *di.it_dev + di.it_off;
        b = beta_at<T>(i);
        first = i == 1;
    }
    // explicit fused multiply-adds (the same in k_rev_combine_mask: the same bits)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const T yb = fma(-tau, gbar[e], vbar[e]);
        if (first) {
            zbar[e] = yb + zbarm[e];
        } else {
            zbar[e] = fma(T(1) + b, yb, zbarm[e]);
            zbarm[e] = -b * yb;
        }
    }
}

// k_rev_combine of iteration i followed, element by element, by k_rev_mask of
// iteration i-1 (z = z(i-1)): the same operations in the same order as the
// two launches, so the same bits.  Elements of the sk2 x sk1 block at the top
// left of each plane (rows of `pitch` values) are skipped (the coarse kernel
// treats them); sk1 = 0: none.
template <typename T>
__global__ void k_rev_combine_mask(T *vbar, const T *gbar, T *zbar, T *zbarm, const T *z, T *wbar, T tau, T b,
                                   int first, int64_t n, DevIter di, int sk1, int sk2, int pitch, int64_t plane)
{
    if (di.it_dev) {
        const int i = *di.it_dev + di.it_off;
        b = beta_at<T>(i);
        first = i == 1;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (sk1 > 0) {
            const int64_t q = e % plane;
            if (q / pitch < sk2 && q % pitch < sk1) continue;
        }
        const T yb = fma(-tau, gbar[e], vbar[e]);
        T zb;
        if (first) {
            zb = yb + zbarm[e];
        } else {
            zb = fma(T(1) + b, yb, zbarm[e]);
            zbarm[e] = -b * yb;
        }
        zbar[e] = zb;
        const T zv = z[e];
        const bool act = zv != T(0);
        vbar[e] = act ? zb : T(0);
        if (wbar && act) {
            const T t = tau * zb;
            wbar[e] = wbar[e] - (zv > T(0) ? t : -t);
        }
    }
}

// y += x
template <typename T>
__global__ void k_add(const T *x, T *y, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] += x[e];
}

// Per-coefficient weight map from per-band weights (Mallat layout).
template <typename T>
__global__ void k_expand_weights(T *w, const T *wlev_dev, int n1, int n2, int C, int levels)
{
    const int64_t N = (int64_t)n1 * n2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * C; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = e % N;
        const int r = (int)(q / n1), c = (int)(q - (int64_t)r * n1);
        int band = 0;
        for (int lev = 1; lev <= levels; ++lev)
            if (r >= (n2 >> lev) || c >= (n1 >> lev)) {
                band = levels + 1 - lev;
                break;
            }
        w[e] = wlev_dev[band];
    }
}

template <typename T>
__global__ void k_copy(const T *src, T *dst, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}


// ----------------------------------------------------- kernel entry points --
// Single problem: arguments by value, tile = blockIdx.  Batched: one launch
// covers the tiles of every image of a phase; a workgroup finds its image in
// the prefix table `start` (tiles of image i are [start[i], start[i+1])),
// copies that image's argument block from device memory and applies the
// per-iteration values (momentum, which buffer holds z(i-1), iteration).

// Tile of this workgroup in XCD-aware order.  Workgroups are dealt to the 8
// XCDs round-robin by linear index, so workgroup b (on XCD b % 8) takes tile
// (b % 8) * per + b / 8: each XCD works through one contiguous run of tiles
// and neighbouring tiles share their halos in that XCD's L2.  Returns -1 for
// the padding workgroups of the last run.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int total)
{
    const int b = blockIdx.x, per = (total + NXCD - 1) / NXCD;
    const int t = (b % NXCD) * per + b / NXCD;
    return t < total ? t : -1;
}
__host__ __device__ inline int xcd_grid(int total) { return NXCD * ((total + NXCD - 1) / NXCD); }


template <typename T>
__global__ __launch_bounds__(NT) void k_synth(SynthArgs<T> a)
{
    const T beta = a.di.it_dev ? beta_at<T>(*a.di.it_dev + a.di.it_off) : a.beta;
    const Live<T> lv{a.zc, a.zp, nullptr, beta, T(0), nullptr};
    const int t = xcd_tile(a.tx * a.ty);  // channel = blockIdx.y
    if (t < 0) return;
    synth_body<T>(a, lv, t % a.tx, t / a.tx, blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_synth2(SynthArgs<T> d, SynthArgs<T> u)
{
    const T beta = d.di.it_dev ? beta_at<T>(*d.di.it_dev + d.di.it_off) : d.beta;
    const Live<T> lv{d.zc, d.zp, nullptr, beta, T(0), nullptr};
    const int t = xcd_tile(d.tx * d.ty);  // channel = blockIdx.y
    if (t < 0) return;
    synth2_body<T>(d, u, lv, t % d.tx, t / d.tx, blockIdx.y);
}

// NTS threads per tile: 1024 when the grid has fewer workgroups than CUs
// can hold two of (the three LDS stages then have four waves per SIMD to
// hide their latency instead of one); the same outputs either way.
template <typename T, int NTS>
__global__ __launch_bounds__(NTS) void k_synth3(SynthArgs<T> d, SynthArgs<T> u, SynthArgs<T> v)
{
    const T beta = d.di.it_dev ? beta_at<T>(*d.di.it_dev + d.di.it_off) : d.beta;
    const Live<T> lv{d.zc, d.zp, nullptr, beta, T(0), nullptr};
    const int t = xcd_tile(d.tx * d.ty);  // channel = blockIdx.y
    if (t < 0) return;
    synth3_body<T, NTS>(d, u, v, lv, t % d.tx, t / d.tx, blockIdx.y);
}

template <typename T>
__device__ __forceinline__ Live<T> live_of(const ProxArgs<T> &p, T beta_next)
{
    if (p.di.it_dev) {
        const int i = *p.di.it_dev + p.di.it_off;
        return Live<T>{p.zc, p.zp, p.zn, beta_at<T>(i), beta_at<T>(i + 1), p.slots};
    }
    return Live<T>{p.zc, p.zp, p.zn, p.beta, beta_next, p.slots};
}

template <typename T, int NCH>
__global__ __launch_bounds__(NT) void k_analysis(AnalysisArgs<T> a)
{
    const int t = xcd_tile(a.tx * a.ty);  // channel group = blockIdx.y
    if (t < 0) return;
    analysis_body<T, NCH>(a, live_of<T>(a.p, T(0)), t % a.tx, t / a.tx, blockIdx.y);
}

// 1024 threads per tile (the passes over the region spread over four waves
// per SIMD; 71 VGPRs in FP32, 119 in FP64)
template <typename T>
constexpr int analysis2_threads() { return 4 * NT; }

template <typename T>
__global__ __launch_bounds__(analysis2_threads<T>()) void k_analysis2(AnalysisArgs<T> a, AnalysisArgs<T> e)
{
    const int t = xcd_tile(a.tx * a.ty);  // channel = blockIdx.y
    if (t < 0) return;
    analysis2_body<T, analysis2_threads<T>()>(a, e, live_of<T>(a.p, T(0)), t % a.tx, t / a.tx, blockIdx.y);
}

// The scalar coarse body, specialised for the geometry every large
// power-of-two plane reaches (a CM x CM block, levels down to an 8 x 8 tail):
// 64 x 64 with 3 pass-by-pass levels in FP32, 32 x 32 with 2 in FP64; and
// within it for the full depth (down to 1 x 1) with the operations of every
// middle iteration.
template <typename T>
__device__ __forceinline__ void coarse_scalar(const CoarseArgs<T> &a, const Live<T> &lv, int bz)
{
    constexpr int CM = CGeom<T>::CM, KW = sizeof(T) == 4 ? 3 : 2, NL = sizeof(T) == 4 ? 6 : 5;
    constexpr int ALL = COARSE_ANA | COARSE_PROX | COARSE_SYN;
    static_assert((CM >> KW) * (CM >> KW) <= PD_TAIL_MAX && (CM >> (KW - 1)) * (CM >> (KW - 1)) > PD_TAIL_MAX,
                  "specialised geometry");
    static_assert((CM >> NL) == 1, "full depth");
    if (a.m1 == CM && a.m2 == CM && a.kw == KW && a.tM1 == (CM >> KW) && a.tM2 == (CM >> KW)) {
        if (a.nlev == NL && a.ops == ALL)
            coarse_body<T, 1, false, CM, KW, (CM >> KW), NL, ALL>(a, lv, bz);
        else
            coarse_body<T, 1, false, CM, KW, (CM >> KW)>(a, lv, bz);
    } else {
        coarse_body<T, 1, false>(a, lv, bz);
    }
}

template <typename T>
__global__ __launch_bounds__(NTC) void k_coarse(CoarseArgs<T> a)
{
    coarse_scalar<T>(a, live_of<T>(a.p, a.beta_next), blockIdx.x);
}
// joint colour: all NCH channels in one workgroup
template <typename T, int NCH>
__global__ __launch_bounds__(NTC) void k_coarse_joint(CoarseArgs<T> a)
{
    coarse_body<T, NCH, true>(a, live_of<T>(a.p, a.beta_next), 0);
}

// The joint (group) prox as its own element-wise launch over an m2 x m1
// region of the Mallat plane (the whole plane, or the coarse block), between a
// per-channel plain analysis (coefficients g in a scratch plane at their
// Mallat positions) and the per-channel synthesis of y(i+1): the same formulas
// as the joint branches of the fused kernels.  A grid of at most JP_GROUPS
// workgroups strides over the positions, JP_UNROLL per thread at a time with
// all their loads in flight, so that the statistics need few atomics.
constexpr int JP_UNROLL = 4;
constexpr int JP_GROUPS = 2048;

template <typename T, int NCH>
__global__ __launch_bounds__(NT) void k_jprox(JProxArgs<T> a)
{
    const ProxArgs<T> &p = a.p;
    const Live<T> lv = live_of<T>(p, T(0));
    const int64_t cnt = (int64_t)a.m1 * a.m2;
    double st[2] = {0.0, 0.0};
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t e0 = (int64_t)blockIdx.x * NT + threadIdx.x; e0 < cnt; e0 += JP_UNROLL * stride) {
        T zc[JP_UNROLL][NCH], zp[JP_UNROLL][NCH], g[JP_UNROLL][NCH];
        int64_t gi[JP_UNROLL];
        int band[JP_UNROLL];
#pragma unroll
        for (int u = 0; u < JP_UNROLL; ++u) {
            const int64_t e = e0 + u * stride < cnt ? e0 + u * stride : e0;  // past the end: a repeat, not stored
            const int r = (int)(e / a.m1), c = (int)(e - (int64_t)r * a.m1);
            int inside = 0;
            for (int lev = 0; lev < a.nlev; ++lev)  // uniform trip count
                inside += (r < (a.m2 >> (lev + 1))) & (c < (a.m1 >> (lev + 1)));
            band[u] = inside == a.nlev ? 0 : a.band_top - inside;
            gi[u] = (int64_t)r * p.pitch + c;
#pragma unroll
            for (int cc = 0; cc < NCH; ++cc) {
                zc[u][cc] = lv.zc[(int64_t)cc * p.plane + gi[u]];
                zp[u][cc] = lv.zp[(int64_t)cc * p.plane + gi[u]];
                g[u][cc] = a.g[(int64_t)cc * p.plane + gi[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < JP_UNROLL; ++u) {
            if (e0 + u * stride >= cnt) continue;
            T w = p.wlev[0];
#pragma unroll
            for (int k = 1; k <= PD_MAXL; ++k) w = band[u] == k ? p.wlev[k] : w;  // selects, no per-lane argument load
            T yv[NCH], vv[NCH];
            T nv = T(0);
            double ny = 0.0;
#pragma unroll
            for (int cc = 0; cc < NCH; ++cc) {
                yv[cc] = momentum(zc[u][cc], zp[u][cc], lv.beta);
                vv[cc] = grad_step(yv[cc], g[u][cc], p.tau);
                nv = fma(vv[cc], vv[cc], nv);
                ny += (double)yv[cc] * (double)yv[cc];
            }
            T nrm = sqrt(nv);
            T sc = nrm > T(0) ? T(1) - p.tau * w / nrm : T(0);
            sc = sc > T(0) ? sc : T(0);
            bad |= !isfinite(nrm);
            st[0] += (double)w * sqrt(ny);
#pragma unroll
            for (int cc = 0; cc < NCH; ++cc) {
                T z = mul_rn(vv[cc], sc);
                lv.zn[(int64_t)cc * p.plane + gi[u]] = z;
                if (p.zsave) p.zsave[(int64_t)cc * p.plane + gi[u]] = z;
                st[1] += ((double)z - (double)yv[cc]) * ((double)z - (double)yv[cc]);
            }
        }
    }
    if (bad) atomicOr(p.flag, 1);
    if (lv.slots) block_slot_add<2, NT>(st, lv.slots + PD_NSLOT);
}

template <typename T, int BT2>
__global__ __launch_bounds__((blur_threads<T, BT2>())) void k_blur(BlurArgs<T> a)
{
    const int t = xcd_tile(a.tx * a.ty);  // channel = blockIdx.y
    if (t < 0) return;
    blur_tile<T, BT2>(a, t % a.tx, t / a.tx, blockIdx.y);
}

// ===========================================================================
// The blur as two marching kernels (large planes).  The same four passes as
// the tile kernel, every output the same sum in the same order, so results
// agree with it bit for bit and the autotuner may pick either:
//   k_blur_h : t = rows of x with the row's own profile, r = columns of t with
//              the source rows' profiles, minus f0           x, f0 -> r
//   k_blur_ht: u = columns of r with the output row's profile, s = rows of u
//              with the same profile                         r -> s
// A wave owns a strip of 128 columns (two neighbouring columns per lane) and
// walks down a block of rows.  Each column pass keeps the last 2R+1 rows of
// its input in registers (a sliding window: nothing is recomputed along x2
// but the first 2R rows of t, and the columns need no LDS); each row pass
// trades one row through a wave-private LDS row.  Profiles are wave-uniform:
// they come from two per-row tables (the own profile, and the profiles
// gathered by output row) through scalar loads.  Waves are independent; the
// workgroup only shares the statistics reduction.
// ===========================================================================
constexpr int TABP = 2 * RM + 2;            // table pitch (taps d = -RM..RM, one pad)
constexpr int SWS = 128;                    // strip width: columns of t, r, u
constexpr int SOT = SWS - 2 * RM - 2;       // s columns per k_blur_ht strip (108, even)
constexpr int NWS = 4;                      // waves per workgroup
constexpr int WIN = 2 * RM + 1;             // window rows
constexpr int SPF = 4;                      // rows loaded ahead of use
constexpr int SRW = SWS + 2 * RM + 6;       // LDS row: columns c0-RM-1 .. c0+SWS+RM (+ pad to 16 bytes)
static_assert(TABP % 4 == 0 && SRW % 4 == 0, "16-byte LDS rows");

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
    T a, b;
};
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
    T v[4];
};

// Orders a wave's LDS writes before the reads of other lanes.  LDS
// operations of one wave execute in order, so only the compiler has to be
// kept from moving memory operations across this point (a plain load may be
// moved across a fence, not across a memory clobber).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// tab[0][p][i]: profile of row p at d = i - RM; tab[1][p][i]: profile of row
// p - d at d (the taps output row p of H gathers); zero where |d| > R.
template <typename T>
__global__ void k_blur_tables(const T *__restrict__ taps, int n2, int R, T *__restrict__ tab)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n2 * TABP) return;
    const int p = e / TABP, i = e - p * TABP, d = i - RM;
    const int W = 2 * R + 1;
    const bool ok = i < WIN && d >= -R && d <= R;
    T own = T(0), gat = T(0);
    if (ok) {
        own = taps[(int64_t)p * W + d + R];
        gat = taps[(int64_t)wrap(p - d, n2) * W + d + R];
    }
    tab[e] = own;
    tab[(int64_t)n2 * TABP + e] = gat;
}

// (strip, row block) of this wave, strips of `width` columns and blocks of
// `rows` rows; workgroups in XCD-aware order (tx workgroups of items).
__device__ __forceinline__ bool march_item(int width, int n1, int n2, int rows, int t, int &c0, int &p0, int &np)
{
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nblk = (n2 + rows - 1) / rows, items = ((n1 + width - 1) / width) * nblk;
    const int item = t * NWS + wv;
    if (t < 0 || item >= items) return false;
    const int strip = item / nblk, blk = item - strip * nblk;
    c0 = strip * width;
    p0 = blk * rows;
    np = n2 - p0 < rows ? n2 - p0 : rows;
    return true;
}

// Copies table rows into the wave's LDS: local row q < na is row
// wrap(pa + q) of table A, local row na + q (q < nb) is row pb + q of table B.
template <typename T>
__device__ __forceinline__ void stage_taps(const T *A, int pa, int na, const T *B, int pb, int nb, int n2, T *dst,
                                           int lane)
{
    constexpr int CPR = TABP / 4;  // 16-byte chunks per row
    const int total = (na + nb) * CPR;
    for (int e0 = 0; e0 < total; e0 += 4 * 64) {
        Quad<T> v[4];
        int at[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // four loads in flight per lane
            const int e = e0 + u * 64 + lane;
            const int ee = e < total ? e : 0;
            const int q = ee / CPR, c = ee - q * CPR;
            const T *src = q < na ? A + (int64_t)wrap(pa + q, n2) * TABP : B + (int64_t)(pb + q - na) * TABP;
            v[u] = reinterpret_cast<const Quad<T> *>(src)[c];
            at[u] = e < total ? q * TABP + 4 * c : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (at[u] >= 0) *reinterpret_cast<Quad<T> *>(dst + at[u]) = v[u];
    }
}

// The 2 RM + 1 taps of one LDS table row (wave-uniform address: broadcast reads).
template <typename T>
__device__ __forceinline__ void read_taps(const T *row, T (&k)[TABP])
{
#pragma unroll
    for (int c = 0; c < TABP / 4; ++c) {
        const Quad<T> q = reinterpret_cast<const Quad<T> *>(row)[c];
#pragma unroll
        for (int u = 0; u < 4; ++u) k[4 * c + u] = q.v[u];
    }
}

// 2 RM + 4 values lrow[2 lane .. 2 lane + 2 RM + 3] as aligned pairs (one
// 2-element vector read each: consecutive lanes read consecutive pairs).
template <typename T>
__device__ __forceinline__ void read_row(const T *lrow, int lane, T (&v)[2 * RM + 4])
{
    typedef T V2 __attribute__((ext_vector_type(2)));
    const V2 *p = reinterpret_cast<const V2 *>(__builtin_assume_aligned(lrow, 2 * sizeof(T)));
#pragma unroll
    for (int i = 0; i < RM + 2; ++i) {
        const V2 q = p[lane + i];
        v[2 * i] = q.x;
        v[2 * i + 1] = q.y;
    }
}

// LDS elements per wave: k_blur_h row (+ for LDS taps: own taps of the steps
// padded to whole blocks of WIN plus one, gathered taps of the rows); k_blur_ht
// row + own taps of the output rows.
__host__ __device__ constexpr int pad_steps(int rows) { return (rows + 2 * RM + WIN - 1) / WIN * WIN; }
template <typename T>
__host__ __device__ constexpr int blur_h_lds(int rows)
{
    return SRW + (sizeof(T) == 4 ? 0 : (pad_steps(rows) + 1 + rows) * TABP);
}
__host__ __device__ constexpr int blur_ht_lds(int rows) { return SRW + rows * TABP; }

// f(integral_constant<int, K>) for K = 0 .. N-1, in order (compile-time slots).
template <typename F, int... K>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, K...>)
{
    (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Row counter that walks down the periodic plane one row per step.
__device__ __forceinline__ int next_row(int r, int n) { return r + 1 == n ? 0 : r + 1; }

// Taps of one table row: FP32 rows come through scalar loads (wave-uniform
// addresses; the values stay in scalar registers), FP64 rows from the
// wave's LDS copy.
template <typename T>
using CT = const __attribute__((address_space(4))) T;
template <typename T>
constexpr bool scalar_taps() { return sizeof(T) == 4; }

template <typename T>
__device__ __forceinline__ void load_taps(const T *gtab, const T *ltab, int grow, int lrow_, T (&k)[TABP])
{
    if constexpr (scalar_taps<T>()) {
        CT<T> *row = (CT<T> *)(gtab + (int64_t)grow * TABP);
#pragma unroll
        for (int i = 0; i < TABP; ++i) k[i] = row[i];
    } else {
        read_taps<T>(ltab + lrow_ * TABP, k);
    }
}

// Steps run in unconditional blocks of WIN (the window slot of step j is
// j mod WIN, and prefetched rows rotate without control flow, so no load in
// flight is ever copied); steps past the block's last row compute values
// that are not stored.  The first block (the warm-up of the column pass) is
// peeled so that its conditions are static.  The next step's taps are
// requested once this step's LDS data has arrived.
template <typename T>
__device__ __forceinline__ void blur_h_body(const BlurArgs<T> &a, int tile, int64_t ch)
{
    extern __shared__ __align__(16) unsigned char blur_lds[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n1 = a.n1, n2 = a.n2;
    double st[1] = {0.0};
    int c0, p0, np;
    if (march_item(SWS, n1, n2, a.rows, tile, c0, p0, np)) {
        const T *x = a.x + ch * a.plane;
        const T *f0 = a.f0 ? a.f0 + ch * a.plane : x;
        T *r = a.r + ch * a.plane;
        T *racc = a.racc ? a.racc + ch * a.plane : nullptr;
        const T *gown = a.tabs, *ggat = a.tabs + (int64_t)n2 * TABP;
        T *lrow = reinterpret_cast<T *>(blur_lds) + wv * blur_h_lds<T>(a.rows);
        const int nsteps = np + 2 * RM;  // t rows p0-RM .. p0+np-1+RM
        const int nblk = (nsteps + WIN - 1) / WIN;
        T *ltown = lrow + SRW;                 // (LDS taps) own profile of t row p0-RM+j at ltown[j]
        T *ltgat = ltown + (nblk * WIN + 1) * TABP;  // gathered taps of r row p0+q at ltgat[q]
        if constexpr (!scalar_taps<T>())
            stage_taps<T>(gown, p0 - RM, nblk * WIN + 1, ggat, p0, np, n2, ltown, lane);
        // LDS slot q holds x column c0-RM-1+q: lanes store slots 2 lane, 2 lane+1
        // and (10 lanes) SWS + 2 lane, +1.  Columns come in even-aligned pairs.
        const int qa = wrap(c0 - RM - 1 + 2 * lane, n1);
        const bool hb = lane < (2 * RM + 2) / 2;
        const int qb = wrap(c0 - RM - 1 + SWS + (hb ? 2 * lane : 0), n1);
        const int cr = c0 + 2 * lane;  // this lane's r columns cr, cr + 1
        const bool own = cr < n1;      // n1 is even: both or neither
        const int crl = own ? cr : 0;
        int xrow = wrap(p0 - RM, n2), frow = wrap(p0 - 2 * RM, n2);  // rows of the next loads
        int trow = xrow;                                              // own-profile row of the next taps
        Pair<T> xa[SPF], xb[SPF], fq[SPF];
        auto load_next = [&](Pair<T> &va, Pair<T> &vb, Pair<T> &vf) {
            const T *rowp = x + (int64_t)xrow * n1;
            va = *reinterpret_cast<const Pair<T> *>(rowp + qa);
            vb = *reinterpret_cast<const Pair<T> *>(rowp + qb);
            vf = *reinterpret_cast<const Pair<T> *>(f0 + (int64_t)frow * n1 + crl);
            xrow = next_row(xrow, n2);
            frow = next_row(frow, n2);
        };
#pragma unroll
        for (int q = 0; q < SPF; ++q) load_next(xa[q], xb[q], fq[q]);
        T kt[TABP], kg[TABP];  // taps of the current step (t pass, r pass)
        load_taps<T>(gown, ltown, trow, 0, kt);
        trow = next_row(trow, n2);
        // gathered taps of r row p0+q into kg (scalar taps; padded steps repeat
        // the block's last row)
        auto load_gat = [&](int q) {
            q = q < np - 1 ? q : np - 1;
            load_taps<T>(ggat, ltgat, p0 + q, q, kg);
        };
        T win[WIN][2];
        if constexpr (!scalar_taps<T>()) wave_lds_sync();  // the staged taps
        const int pend = p0 + np;
        // step j in window slot k: t of row p0-RM+j; with_r: r of row p0+j-2RM
        auto step = [&](int j, auto kc, auto rc, auto nc) {
            constexpr int k = decltype(kc)::value;
            constexpr bool with_r = decltype(rc)::value, next_r = decltype(nc)::value;
            const Pair<T> cx = xa[0], cxb = xb[0], cf = fq[0];
#pragma unroll
            for (int q = 0; q + 1 < SPF; ++q) {
                xa[q] = xa[q + 1];
                xb[q] = xb[q + 1];
                fq[q] = fq[q + 1];
            }
            load_next(xa[SPF - 1], xb[SPF - 1], fq[SPF - 1]);
            *reinterpret_cast<Pair<T> *>(lrow + 2 * lane) = cx;
            if (hb) *reinterpret_cast<Pair<T> *>(lrow + SWS + 2 * lane) = cxb;
            wave_lds_sync();
            T xs[2 * RM + 4];
            read_row<T>(lrow, lane, xs);  // xs[i] = x column cr - RM - 1 + i
            wave_lds_sync();
            // t of row p0-RM+j: rows pass with the row's own profile
            T t0 = T(0), t1 = T(0);
#pragma unroll
            for (int m = 0; m <= 2 * RM; ++m) {
                const T kk = kt[2 * RM - m];  // d = RM - m: t(c) = sum k[d] x(c - d)
                t0 = fma(kk, xs[m + 1], t0);
                t1 = fma(kk, xs[m + 2], t1);
            }
            // computed here, not sunk towards the (later) column pass: bounded lifetimes
            __asm__ __volatile__("" : "+v"(t0), "+v"(t1));
            win[k][0] = t0;
            win[k][1] = t1;
            load_taps<T>(gown, ltown, trow, j + 1, kt);  // the next step's own profile
            trow = next_row(trow, n2);
            T kr[TABP];  // this step's gathered taps
            if constexpr (scalar_taps<T>()) {
#pragma unroll
                for (int i = 0; i < TABP; ++i) kr[i] = kg[i];
                if (next_r) load_gat(j + 1 - 2 * RM);  // the next step's, requested early
                __builtin_amdgcn_sched_barrier(0);     // (not sunk into the next step)
            } else if (with_r) {
                const int q = j - 2 * RM < np - 1 ? j - 2 * RM : np - 1;
                read_taps<T>(ltgat + q * TABP, kr);
            }
            if (with_r) {
                // columns of t with the source rows' profiles, d = -RM..RM
                // (t row p-d sits in slot (k + d - RM) mod WIN)
                T r0 = T(0), r1 = T(0);
#pragma unroll
                for (int i = 0; i <= 2 * RM; ++i) {
                    const int sl = (k - i + 2 * WIN) % WIN;
                    r0 = fma(kr[i], win[sl][0], r0);
                    r1 = fma(kr[i], win[sl][1], r1);
                }
                r0 = r0 - (a.f0 ? cf.a : T(0));
                r1 = r1 - (a.f0 ? cf.b : T(0));
                const int pr = p0 + j - 2 * RM;
                if (own && pr < pend) {
                    const int64_t o = (int64_t)pr * n1 + cr;
                    *reinterpret_cast<Pair<T> *>(r + o) = Pair<T>{r0, r1};
                    st[0] += 0.5 * (double)r0 * (double)r0;
                    st[0] += 0.5 * (double)r1 * (double)r1;
                    if (racc) {
                        racc[o] = fma(a.rscale, r0, racc[o]);
                        racc[o + 1] = fma(a.rscale, r1, racc[o + 1]);
                    }
                }
            }
        };
        static_for<WIN>([&](auto kc) {  // warm-up block
            constexpr int k = decltype(kc)::value;
            step(k, kc, std::integral_constant<bool, (k >= 2 * RM)>{}, std::integral_constant<bool, (k + 1 >= 2 * RM)>{});
        });
        for (int base = WIN; base < nsteps; base += WIN)
            static_for<WIN>([&](auto kc) {
                step(base + decltype(kc)::value, kc, std::true_type{}, std::true_type{});
            });
    }
    if (a.slots) block_slot_add<1, 64 * NWS>(st, a.slots);
}

// tile = the workgroup's index among the tx of a channel; ch its channel
template <typename T>
__global__ __launch_bounds__(64 * NWS) void k_blur_h(BlurArgs<T> a)
{
    const int t = xcd_tile(a.tx);
    if (t < 0) return;  // padding workgroup (uniform)
    blur_h_body<T>(a, t, blockIdx.y);
}

// The H^T kernel reads its taps from the wave's LDS copy (one profile per
// step, needed at the start of the step).
template <typename T>
__device__ __forceinline__ void blur_ht_body(const BlurArgs<T> &a, int tile, int64_t ch)
{
    extern __shared__ __align__(16) unsigned char blur_lds[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n1 = a.n1, n2 = a.n2;
    int c0, p0, np;
    if (!march_item(SOT, n1, n2, a.rows, tile, c0, p0, np)) return;
    const T *rin = a.r + ch * a.plane;
    T *s = a.s + ch * a.plane;
    T *lrow = reinterpret_cast<T *>(blur_lds) + wv * blur_ht_lds(a.rows);
    T *ltown = lrow + SRW;  // own profile of output row p0+q at ltown[q]
    stage_taps<T>(a.tabs, p0, np, a.tabs, 0, 0, n2, ltown, lane);
    // u columns (LDS slots 2 lane, 2 lane+1) = r columns c0-RM-1+2 lane, +1;
    // s columns c0 + 2 lane, +1 for the first SOT/2 lanes
    const int qu = wrap(c0 - RM - 1 + 2 * lane, n1);
    const int cs = c0 + 2 * lane;
    const bool own = lane < SOT / 2 && cs < n1;
    const int nsteps = np + 2 * RM;  // r rows p0-RM .. p0+np-1+RM enter the window
    int rrow = wrap(p0 - RM, n2);
    Pair<T> rq[SPF];
    auto load_next = [&](Pair<T> &v) {
        v = *reinterpret_cast<const Pair<T> *>(rin + (int64_t)rrow * n1 + qu);
        rrow = next_row(rrow, n2);
    };
#pragma unroll
    for (int q = 0; q < SPF; ++q) load_next(rq[q]);
    T win[WIN][2];
    wave_lds_sync();  // the staged taps
    const int pend = p0 + np;
    auto step = [&](int j, auto kc, auto uc) {
        constexpr int k = decltype(kc)::value;
        constexpr bool with_u = decltype(uc)::value;
        win[k][0] = rq[0].a;
        win[k][1] = rq[0].b;
#pragma unroll
        for (int q = 0; q + 1 < SPF; ++q) rq[q] = rq[q + 1];
        load_next(rq[SPF - 1]);
        if (with_u) {
            // the output row's profile (padded steps repeat the block's last row)
            const int q = j - 2 * RM < np - 1 ? j - 2 * RM : np - 1;
            T kp[TABP];
            read_taps<T>(ltown + q * TABP, kp);
            // u of row p: r rows p+d (d = -RM..RM) sit in slots (k + 1 + i) mod WIN, i = d + RM
            T u0 = T(0), u1 = T(0);
#pragma unroll
            for (int i = 0; i <= 2 * RM; ++i) {
                const int sl = (k + 1 + i) % WIN;
                u0 = fma(kp[i], win[sl][0], u0);
                u1 = fma(kp[i], win[sl][1], u1);
            }
            *reinterpret_cast<Pair<T> *>(lrow + 2 * lane) = Pair<T>{u0, u1};
            wave_lds_sync();
            T us[2 * RM + 4];
            read_row<T>(lrow, lane, us);  // us[i] = u column cs - RM - 1 + i
            wave_lds_sync();
            // s(c) = sum_{m} k[m - RM] u(c - RM + m), m = 0..2RM
            T s0 = T(0), s1 = T(0);
#pragma unroll
            for (int m = 0; m <= 2 * RM; ++m) {
                s0 = fma(kp[m], us[m + 1], s0);
                s1 = fma(kp[m], us[m + 2], s1);
            }
            const int pr = p0 + j - 2 * RM;
            if (own && pr < pend) *reinterpret_cast<Pair<T> *>(s + (int64_t)pr * n1 + cs) = Pair<T>{s0, s1};
        }
    };
    static_for<WIN>([&](auto kc) {  // warm-up block: the window fills
        constexpr int k = decltype(kc)::value;
        step(k, kc, std::integral_constant<bool, (k >= 2 * RM)>{});
    });
    for (int base = WIN; base < nsteps; base += WIN)
        static_for<WIN>([&](auto kc) { step(base + decltype(kc)::value, kc, std::true_type{}); });
}

template <typename T>
__global__ __launch_bounds__(64 * NWS) void k_blur_ht(BlurArgs<T> a)
{
    const int t = xcd_tile(a.tx);
    if (t < 0) return;
    blur_ht_body<T>(a, t, blockIdx.y);
}

__device__ __forceinline__ int locate(const int *__restrict__ start, int n, int blk)
{
    int lo = 0, hi = n;  // start[lo] <= blk < start[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (start[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Live values of a batched iteration: the table holds z(0) in zc and its copy
// in zp; odd iterations swap them, z(i) goes in place of z(i-2).
template <typename T>
__device__ __forceinline__ Live<T> live_dyn(const ProxArgs<T> &p, const Dyn<T> &d)
{
    const T *zc = d.parity ? p.zp : p.zc, *zp = d.parity ? p.zc : p.zp;
    return Live<T>{zc, zp, const_cast<T *>(zp), d.beta, d.beta_next,
                   p.slots ? p.slots + (size_t)d.ring * 3 * PD_NSLOT : nullptr};
}

// Momenta of a replayed launch from the device iteration number.
template <typename T>
__device__ __forceinline__ Dyn<T> dyn_at(Dyn<T> d)
{
    if (d.it_dev) {
        const int i = *d.it_dev + d.it_off;
        d.beta = beta_at<T>(i);
        d.beta_next = beta_at<T>(i + 1);
    }
    return d;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_synth_b(const SynthArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                 int n, Dyn<T> d)
{
    d = dyn_at<T>(d);
    const int g = xcd_tile(start[n]);
    if (g < 0) return;
    const int img = locate(start, n, g);
    const SynthArgs<T> &a = tab[img];
    const Live<T> lv{d.parity ? a.zp : a.zc, d.parity ? a.zc : a.zp, nullptr, d.beta, T(0), nullptr};
    int loc = g - start[img];
    const int tx = a.tx, ty = a.ty;
    const int bx = loc % tx;
    loc /= tx;
    synth_body<T>(a, lv, bx, loc % ty, loc / ty);
}

// NCH = 0: scalar prox, one tile set per channel; NCH >= 1: joint prox over
// NCH channels per tile (every image of the launch has NCH channels).
template <typename T, int NCH>
__global__ __launch_bounds__(NT) void k_analysis_b(const AnalysisArgs<T> *__restrict__ tab,
                                                    const int *__restrict__ start, int n, Dyn<T> d)
{
    d = dyn_at<T>(d);
    const int g = xcd_tile(start[n]);
    if (g < 0) return;
    const int img = locate(start, n, g);
    const AnalysisArgs<T> &a = tab[img];
    const Live<T> lv = a.mode == MODE_PROX ? live_dyn<T>(a.p, d) : live_of<T>(a.p, T(0));
    int loc = g - start[img];
    const int tx = a.tx, ty = a.ty;
    const int bx = loc % tx;
    loc /= tx;
    analysis_body<T, NCH>(a, lv, bx, loc % ty, loc / ty);
}

// NCH as for the joint coarse kernel: 1 with one workgroup per channel (scalar
// prox), or the channel count of joint images (one workgroup per image).
template <typename T, int NCH, bool JOINT>
__global__ __launch_bounds__(NTC) void k_coarse_b(const CoarseArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                   int n, Dyn<T> d)
{
    d = dyn_at<T>(d);
    const int img = locate(start, n, blockIdx.x);
    const CoarseArgs<T> &a = tab[img];
    Live<T> lv;
    if (a.ops & COARSE_PROX) {
        lv = live_dyn<T>(a.p, d);
    } else if (!(a.ops & COARSE_ANA)) {  // synthesis only: y from the state
        lv = live_dyn<T>(a.p, d);
        lv.slots = nullptr;
    } else {
        lv = live_of<T>(a.p, T(0));
    }
    if constexpr (!JOINT && NCH == 1)
        coarse_scalar<T>(a, lv, blockIdx.x - start[img]);
    else
        coarse_body<T, NCH, JOINT>(a, lv, JOINT ? 0 : blockIdx.x - start[img]);
}

template <typename T>
__global__ __launch_bounds__((blur_threads<T, 32>())) void k_blur_b(const BlurArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                int n, int ring)
{
    const int g = xcd_tile(start[n]);
    if (g < 0) return;
    const int img = locate(start, n, g);
    BlurArgs<T> a = tab[img];
    if (a.slots) a.slots += (size_t)ring * 3 * PD_NSLOT;
    int loc = g - start[img];
    const int bx = loc % a.tx;
    loc /= a.tx;
    blur_tile<T, 32>(a, bx, loc % a.ty, loc / a.ty);
}

// The two marching kernels over many images: workgroup g of the launch is
// tile (g - start[img]) % tx of channel (g - start[img]) / tx of its image
// (tx = the image's workgroups per channel, a different count for each kernel).
template <typename T>
__global__ __launch_bounds__(64 * NWS) void k_blur_h_b(const BlurArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                       int n, int ring)
{
    const int g = xcd_tile(start[n]);
    if (g < 0) return;
    const int img = locate(start, n, g);
    BlurArgs<T> a = tab[img];
    if (a.slots) a.slots += (size_t)ring * 3 * PD_NSLOT;
    const int loc = g - start[img];
    blur_h_body<T>(a, loc % a.tx, loc / a.tx);
}

template <typename T>
__global__ __launch_bounds__(64 * NWS) void k_blur_ht_b(const BlurArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                        int n)
{
    const int g = xcd_tile(start[n]);
    if (g < 0) return;
    const int img = locate(start, n, g);
    const BlurArgs<T> &a = tab[img];
    const int loc = g - start[img];
    blur_ht_body<T>(a, loc % a.ty, loc / a.ty);  // (ty holds the H^T kernel's workgroups per channel)
}

// ------------------------------------------------------------ launchers ---
template <typename T>
hipError_t launch_synth2(const SynthArgs<T> &d, const SynthArgs<T> &u, int C, hipStream_t s)
{
    SynthArgs<T> b = d;
    tiles_synth(d.M1c, d.M2c, &b.tx, &b.ty);
    hipLaunchKernelGGL(k_synth2<T>, dim3(xcd_grid(b.tx * b.ty), C), dim3(NT), 0, s, b, u);
    return hipGetLastError();
}

constexpr int SYNTH3_WIDE_BELOW = 512;  // workgroups: two per CU

template <typename T>
hipError_t launch_synth3(const SynthArgs<T> &d, const SynthArgs<T> &u, const SynthArgs<T> &v, int C, hipStream_t s)
{
    SynthArgs<T> b = d;
    tiles_synth(d.M1c, d.M2c, &b.tx, &b.ty);
    if (b.tx * b.ty * C < SYNTH3_WIDE_BELOW)
        hipLaunchKernelGGL((k_synth3<T, 4 * NT>), dim3(xcd_grid(b.tx * b.ty), C), dim3(4 * NT), 0, s, b, u, v);
    else
        hipLaunchKernelGGL((k_synth3<T, NT>), dim3(xcd_grid(b.tx * b.ty), C), dim3(NT), 0, s, b, u, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_synth(const SynthArgs<T> &a, int C, hipStream_t s)
{
    SynthArgs<T> b = a;
    tiles_synth(a.M1c, a.M2c, &b.tx, &b.ty);
    hipLaunchKernelGGL(k_synth<T>, dim3(xcd_grid(b.tx * b.ty), C), dim3(NT), 0, s, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_analysis2(const AnalysisArgs<T> &a, const AnalysisArgs<T> &e, hipStream_t s)
{
    if (a.p.joint || e.M1c * 2 != a.M1c || e.M2c * 2 != a.M2c || a.last || e.mode != a.mode)
        return hipErrorInvalidValue;
    AnalysisArgs<T> b = a;
    tiles_analysis(a.M1c, a.M2c, &b.tx, &b.ty);
    hipLaunchKernelGGL(k_analysis2<T>, dim3(xcd_grid(b.tx * b.ty), a.p.C), dim3(analysis2_threads<T>()), 0, s, b,
                       e);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_analysis(const AnalysisArgs<T> &a, hipStream_t s)
{
    AnalysisArgs<T> b = a;
    tiles_analysis(a.M1c, a.M2c, &b.tx, &b.ty);
    const int groups = a.p.joint ? 1 : a.p.C;
    dim3 grid(xcd_grid(b.tx * b.ty), groups);
    if (!a.p.joint)
        hipLaunchKernelGGL((k_analysis<T, 0>), grid, dim3(NT), 0, s, b);
    else if (a.p.C == 1)  // (several channels: plain analysis + k_jprox)
        hipLaunchKernelGGL((k_analysis<T, 1>), grid, dim3(NT), 0, s, b);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
size_t coarse_lds_bytes(int m1, int m2, int chans)
{
    if (m1 > CGeom<T>::CM || m2 > CGeom<T>::CM) return SIZE_MAX;
    return sizeof(T) * (size_t)CLayout<T>(m1, m2, chans).total;
}

template <typename T>
hipError_t launch_jprox(const JProxArgs<T> &a, int nch, hipStream_t s)
{
    const int64_t cnt = (int64_t)a.m1 * a.m2;
    const int64_t want = (cnt + JP_UNROLL * NT - 1) / (JP_UNROLL * NT);
    const int groups = want < JP_GROUPS ? (int)want : JP_GROUPS;
    const dim3 grid(groups > 0 ? groups : 1);
    switch (nch) {
    case 1: hipLaunchKernelGGL((k_jprox<T, 1>), grid, dim3(NT), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_jprox<T, 2>), grid, dim3(NT), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_jprox<T, 3>), grid, dim3(NT), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_jprox<T, 4>), grid, dim3(NT), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse(const CoarseArgs<T> &a, int groups, hipStream_t s)
{
    const int chans = a.p.joint ? a.p.C : 1;
    size_t lds = coarse_lds_bytes<T>(a.m1, a.m2, chans);
    if (!a.p.joint)
        hipLaunchKernelGGL(k_coarse<T>, dim3(groups), dim3(NTC), lds, s, a);
    else if (chans == 1)  // (several channels: per-channel analysis/synthesis + k_jprox)
        hipLaunchKernelGGL((k_coarse_joint<T, 1>), dim3(groups), dim3(NTC), lds, s, a);
    else
        return hipErrorInvalidValue;
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
        BlurArgs<T> b = a;
        const int v = blur_variant(a.n1, a.n2, a.C, a.R, (int)sizeof(T));
        if (v > BLUR_SPLIT && a.r && a.tabs) {
            b.rows = v - BLUR_SPLIT;
            const int nb = (a.n2 + b.rows - 1) / b.rows;
            b.tx = ((a.n1 + SWS - 1) / SWS * nb + NWS - 1) / NWS;
            hipLaunchKernelGGL(k_blur_h<T>, dim3(xcd_grid(b.tx), a.C), dim3(64 * NWS),
                               NWS * blur_h_lds<T>(b.rows) * sizeof(T), s, b);
            b.tx = ((a.n1 + SOT - 1) / SOT * nb + NWS - 1) / NWS;
            hipLaunchKernelGGL(k_blur_ht<T>, dim3(xcd_grid(b.tx), a.C), dim3(64 * NWS),
                               NWS * blur_ht_lds(b.rows) * sizeof(T), s, b);
            return hipGetLastError();
        }
        const int bt2 = v == 48 ? 48 : 32;
        tiles_blur(a.n1, a.n2, &b.tx, &b.ty, bt2);
        if (bt2 == 48)
            hipLaunchKernelGGL((k_blur<T, 48>), dim3(xcd_grid(b.tx * b.ty), a.C), dim3(blur_threads<T, 48>()), 0, s,
                               b);
        else
            hipLaunchKernelGGL((k_blur<T, 32>), dim3(xcd_grid(b.tx * b.ty), a.C), dim3(blur_threads<T, 32>()), 0, s,
                               b);
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

template <typename T>
hipError_t launch_synth_b(const SynthArgs<T> *tab, const int *start, int n, int tiles, Dyn<T> d, hipStream_t s)
{
    hipLaunchKernelGGL(k_synth_b<T>, dim3(xcd_grid(tiles)), dim3(NT), 0, s, tab, start, n, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_analysis_b(const AnalysisArgs<T> *tab, const int *start, int n, int tiles, int nch, Dyn<T> d,
                             hipStream_t s)
{
    const dim3 grid(xcd_grid(tiles));
    switch (nch) {
    case 0: hipLaunchKernelGGL((k_analysis_b<T, 0>), grid, dim3(NT), 0, s, tab, start, n, d); break;
    case 1: hipLaunchKernelGGL((k_analysis_b<T, 1>), grid, dim3(NT), 0, s, tab, start, n, d); break;
    case 2: hipLaunchKernelGGL((k_analysis_b<T, 2>), grid, dim3(NT), 0, s, tab, start, n, d); break;
    case 3: hipLaunchKernelGGL((k_analysis_b<T, 3>), grid, dim3(NT), 0, s, tab, start, n, d); break;
    case 4: hipLaunchKernelGGL((k_analysis_b<T, 4>), grid, dim3(NT), 0, s, tab, start, n, d); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_b(const CoarseArgs<T> *tab, const int *start, int n, int groups, size_t lds, int nch,
                           Dyn<T> d, hipStream_t s)
{
    switch (nch) {
    case 0: hipLaunchKernelGGL((k_coarse_b<T, 1, false>), dim3(groups), dim3(NTC), lds, s, tab, start, n, d); break;
    case 1: hipLaunchKernelGGL((k_coarse_b<T, 1, true>), dim3(groups), dim3(NTC), lds, s, tab, start, n, d); break;
    case 2: hipLaunchKernelGGL((k_coarse_b<T, 2, true>), dim3(groups), dim3(NTC), lds, s, tab, start, n, d); break;
    case 3: hipLaunchKernelGGL((k_coarse_b<T, 3, true>), dim3(groups), dim3(NTC), lds, s, tab, start, n, d); break;
    case 4: hipLaunchKernelGGL((k_coarse_b<T, 4, true>), dim3(groups), dim3(NTC), lds, s, tab, start, n, d); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Workgroups per channel of the two marching kernels for an n1 x n2 plane, `rows` rows per wave.
void tiles_blur_split(int n1, int n2, int rows, int *th, int *tht)
{
    const int nb = (n2 + rows - 1) / rows;
    *th = ((n1 + SWS - 1) / SWS * nb + NWS - 1) / NWS;
    *tht = ((n1 + SOT - 1) / SOT * nb + NWS - 1) / NWS;
}

template <typename T>
hipError_t launch_blur_split_b(const BlurArgs<T> *tab, const int *start_h, const int *start_ht, int n, int wg_h,
                               int wg_ht, int rows, int ring, hipStream_t s)
{
    hipLaunchKernelGGL(k_blur_h_b<T>, dim3(xcd_grid(wg_h)), dim3(64 * NWS), NWS * blur_h_lds<T>(rows) * sizeof(T), s,
                       tab, start_h, n, ring);
    hipLaunchKernelGGL(k_blur_ht_b<T>, dim3(xcd_grid(wg_ht)), dim3(64 * NWS), NWS * blur_ht_lds(rows) * sizeof(T), s,
                       tab, start_ht, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blur_b(const BlurArgs<T> *tab, const int *start, int n, int tiles, int ring, hipStream_t s)
{
    hipLaunchKernelGGL(k_blur_b<T>, dim3(xcd_grid(tiles)), dim3(blur_threads<T, 32>()), 0, s, tab, start, n, ring);
    return hipGetLastError();
}

hipError_t launch_stats_finalize_b(double *const *ring, double *const *stats, int n, int it0, int count,
                                   const int *it_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_finalize_b, dim3(count, n), dim3(256), 0, s, ring, stats, it0, it_dev);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *dst, T v, int64_t n, hipStream_t s)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, s, dst, v, n);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(double *, double, int64_t, hipStream_t);
template hipError_t launch_fill<float>(float *, float, int64_t, hipStream_t);

static inline int ew_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <typename T>
hipError_t launch_rev_mask(const T *zbar, const T *z, T *vbar, T *wbar, T tau, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_rev_mask<T>, dim3(ew_blocks(n)), dim3(256), 0, s, zbar, z, vbar, wbar, tau, n);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_rev_combine(const T *vbar, const T *gbar, T *zbar, T *zbarm, T tau, T b, int first, int64_t n,
                              DevIter di, hipStream_t s)
{
    hipLaunchKernelGGL(k_rev_combine<T>, dim3(ew_blocks(n)), dim3(256), 0, s, vbar, gbar, zbar, zbarm, tau, b, first, n,
                       di);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_rev_combine_mask(T *vbar, const T *gbar, T *zbar, T *zbarm, const T *z, T *wbar, T tau, T b,
                                   int first, int64_t n, DevIter di, int sk1, int sk2, int pitch, int64_t plane,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_rev_combine_mask<T>, dim3(ew_blocks(n)), dim3(256), 0, s, vbar, gbar, zbar, zbarm, z, wbar,
                       tau, b, first, n, di, sk1, sk2, pitch, plane);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_add(const T *x, T *y, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add<T>, dim3(ew_blocks(n)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_expand_weights(T *w, const T *wlev_dev, int n1, int n2, int C, int levels, hipStream_t s)
{
    hipLaunchKernelGGL(k_expand_weights<T>, dim3(ew_blocks((int64_t)n1 * n2 * C)), dim3(256), 0, s, w, wlev_dev, n1,
                       n2, C, levels);
    return hipGetLastError();
}
#define PD_INST_REV(T)                                                                                  \
    template hipError_t launch_rev_mask<T>(const T *, const T *, T *, T *, T, int64_t, hipStream_t);    \
    template hipError_t launch_rev_combine<T>(const T *, const T *, T *, T *, T, T, int, int64_t, DevIter, \
                                              hipStream_t);                                             \
    template hipError_t launch_rev_combine_mask<T>(T *, const T *, T *, T *, const T *, T *, T, T, int, int64_t, \
                                                   DevIter, int, int, int, int64_t, hipStream_t);                \
    template hipError_t launch_add<T>(const T *, T *, int64_t, hipStream_t);                            \
    template hipError_t launch_expand_weights<T>(T *, const T *, int, int, int, int, hipStream_t);
PD_INST_REV(float)
PD_INST_REV(double)

void tiles_synth(int M1c, int M2c, int *tx, int *ty) { *tx = (M1c + SP - 1) / SP; *ty = (M2c + SP - 1) / SP; }
void tiles_analysis(int M1c, int M2c, int *tx, int *ty) { *tx = (M1c + TC - 1) / TC; *ty = (M2c + TC - 1) / TC; }
// The autotuning cache: the blur variant chosen by pd_tune per
// (n1, n2, channels, radius, element size); the 32-row tile kernel where
// nothing was tuned.
namespace {
std::mutex g_tune_mu;
std::map<std::array<int, 5>, int> g_blur_variant;
}  // namespace

int blur_variant(int n1, int n2, int C, int R, int es)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_blur_variant.find({n1, n2, C, R, es});
    return it == g_blur_variant.end() ? 32 : it->second;
}

void set_blur_variant(int n1, int n2, int C, int R, int es, int v)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_blur_variant[{n1, n2, C, R, es}] = v;
}

template <typename T>
hipError_t launch_blur_tables(const T *taps, int n2, int R, T *tab, hipStream_t s)
{
    const int n = n2 * TABP;
    hipLaunchKernelGGL(k_blur_tables<T>, dim3((n + 255) / 256), dim3(256), 0, s, taps, n2, R, tab);
    return hipGetLastError();
}
template hipError_t launch_blur_tables<float>(const float *, int, int, float *, hipStream_t);
template hipError_t launch_blur_tables<double>(const double *, int, int, double *, hipStream_t);
static_assert(TABP == BLUR_TAB_PITCH, "table pitch");

void tiles_blur(int n1, int n2, int *tx, int *ty, int bt2)
{
    *tx = (n1 + BT1 - 1) / BT1;
    *ty = (n2 + bt2 - 1) / bt2;
}

hipError_t launch_stats_finalize(double *ring, double *stats, int it0, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_finalize, dim3(count), dim3(256), 0, s, ring, stats, it0);
    return hipGetLastError();
}

hipError_t launch_stats_finalize_dev(double *ring, double *stats, const int *it_dev, int sub, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_finalize_dev, dim3(count), dim3(256), 0, s, ring, stats, it_dev, sub);
    return hipGetLastError();
}

hipError_t launch_set_int(int *dst, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

#define PD_INST(T)                                                                          \
    template hipError_t launch_synth<T>(const SynthArgs<T> &, int, hipStream_t);           \
    template hipError_t launch_analysis<T>(const AnalysisArgs<T> &, hipStream_t);          \
    template hipError_t launch_synth2<T>(const SynthArgs<T> &, const SynthArgs<T> &, int, hipStream_t); \
    template hipError_t launch_synth3<T>(const SynthArgs<T> &, const SynthArgs<T> &, const SynthArgs<T> &, int,  \
                                         hipStream_t);                                                         \
    template hipError_t launch_coarse<T>(const CoarseArgs<T> &, int, hipStream_t);         \
    template hipError_t launch_jprox<T>(const JProxArgs<T> &, int, hipStream_t); \
    template size_t coarse_lds_bytes<T>(int, int, int);                                    \
    template hipError_t launch_blur<T>(const BlurArgs<T> &, bool, hipStream_t);            \
    template hipError_t launch_analysis2<T>(const AnalysisArgs<T> &, const AnalysisArgs<T> &, hipStream_t); \
    template hipError_t launch_blur_single<T>(const BlurArgs<T> &, int, hipStream_t);      \
    template hipError_t launch_copy<T>(const T *, T *, int64_t, hipStream_t);                   \
    template hipError_t launch_synth_b<T>(const SynthArgs<T> *, const int *, int, int, Dyn<T>, hipStream_t); \
    template hipError_t launch_analysis_b<T>(const AnalysisArgs<T> *, const int *, int, int, int, Dyn<T>,     \
                                             hipStream_t);                                                      \
    template hipError_t launch_coarse_b<T>(const CoarseArgs<T> *, const int *, int, int, size_t, int, Dyn<T>,  \
                                           hipStream_t);                                                        \
    template hipError_t launch_blur_b<T>(const BlurArgs<T> *, const int *, int, int, int, hipStream_t);        \
    template hipError_t launch_blur_split_b<T>(const BlurArgs<T> *, const int *, const int *, int, int, int, int, \
                                               int, hipStream_t);
PD_INST(float)
PD_INST(double)

}  // namespace pd
