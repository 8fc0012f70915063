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

#include <cstdint>

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
        double a = v[q];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) red[q][wv] = a;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double a = 0.0;
        for (int k = 0; k < NTH / 64; ++k) a += red[threadIdx.x][k];
        const unsigned blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        atomicAdd(slots + threadIdx.x * PD_NSLOT + (blk % PD_NSLOT), a);
    }
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
template <typename T>
__device__ __forceinline__ T prox1(T y, T g, T tau, T w, double (&st)[2], bool &bad)
{
    T v = y - tau * g;
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
__device__ __forceinline__ void synth_body(const SynthArgs<T> &a, int bx, int by, int bz)
{
    __shared__ T sB[4][SR][SR + 1];   // LL, HL (hi x1), LH (hi x2), HH
    __shared__ T sLH[2][SF][SR + 1];  // after x2 synthesis: low / high along x1
    const int M1c = a.M1c, M2c = a.M2c;
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int64_t ch = bz;
    const int p01 = bx * SP, p02 = by * SP;
    const T *zc = a.zc + ch * a.plane;
    const T *zp = a.zp + ch * a.plane;
    const T *apx = a.apx ? a.apx + ch * a.apx_plane : nullptr;
    const int tid = threadIdx.x;

    // load: wave-row R < 26 covers the top bands (LL | HL) of coarse row R,
    // R >= 26 the bottom bands (LH | HH); lanes 0..25 the low-x1 band, 26..51
    // the high-x1 band.  Column offsets are per lane, row bases per wave-row.
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool lok = lane < 2 * SR;
    const bool hi1 = lane >= SR;
    const int lc_ = hi1 ? lane - SR : lane;
    const int q1 = lok ? wrap(p01 - 5 + lc_, M1c) : 0;
    const int col = q1 + (hi1 ? M1c : 0);
    constexpr int RPW = (2 * SR) / (NT / 64);  // 13 wave-rows per wave
    T va[RPW], vb[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int R = wv + i * (NT / 64);
        const bool bottom = R >= SR;
        const int r = bottom ? R - SR : R;
        const int q2 = wrap(p02 - 5 + r, M2c);
        va[i] = T(0);
        vb[i] = T(0);
        if (!lok) continue;
        if (!bottom && !hi1 && apx) {
            va[i] = apx[(int64_t)q2 * M1c + q1];
            vb[i] = va[i];
        } else {
            const int64_t idx = (int64_t)(q2 + (bottom ? M2c : 0)) * a.pitch + col;
            va[i] = zc[idx];
            vb[i] = zp[idx];
        }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int R = wv + i * (NT / 64);
        const bool bottom = R >= SR;
        const int r = bottom ? R - SR : R;
        if (lok) sB[(hi1 ? 1 : 0) + (bottom ? 2 : 0)][r][lc_] = va[i] + a.beta * (va[i] - vb[i]);
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

template <typename T, bool JOINT>
__device__ __forceinline__ void analysis_body(const AnalysisArgs<T> &a, int bx, int by, int bz)
{
    __shared__ T sIn[AR][AR + 4];  // pitch 56: aligned 16-byte reads
    __shared__ T sRow[2][AR][TC + 1];  // low / high along x1
    const int M1c = a.M1c, M2c = a.M2c;
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int c01 = bx * TC, c02 = by * TC;
    const int tid = threadIdx.x;
    const ProxArgs<T> &p = a.p;
    const int nch = JOINT ? p.C : 1;
    const int ch0 = JOINT ? 0 : bz;

    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool lok = lane < AR;
    const int qc = lok ? wrap(2 * c01 - 10 + lane, M1) : 0;
    // column-pass task of this thread: (src band along x1, coarse column, 2 rows)
    const int src = tid / (TC * (TC / 2));
    const int rem = tid - src * (TC * (TC / 2));
    const int rblk = rem / TC, l1 = rem - rblk * TC;
    T res[JOINT ? PD_MAXC : 1][4];  // [ch][ (h, g) x 2 rows ]

    for (int cc = 0; cc < nch; ++cc) {
        const int ch = ch0 + cc;
        const T *in = a.in + (int64_t)ch * a.in_plane;
        // load: lane = fine column (52 of 64 lanes), wave = fine rows
        constexpr int RPW = AR / (NT / 64);  // 13
        T v[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + i * (NT / 64);
            const T *rowp = in + (int64_t)wrap(2 * c02 - 10 + r, M2) * a.in_pitch;
            v[i] = lok ? rowp[qc] : T(0);
        }
        if (JOINT && cc > 0) __syncthreads();  // previous channel's passes are done
#pragma unroll
        for (int i = 0; i < RPW; ++i)
            if (lok) sIn[wv + i * (NT / 64)][lane] = v[i];
        __syncthreads();
        // along x1: task = (fine row r, block of 4 coarse columns)
        for (int t = tid; t < AR * (TC / 4); t += NT) {
            int r = t / (TC / 4), blk = t - r * (TC / 4);
            T x[28];
#pragma unroll
            for (int j = 0; j < 28; ++j) x[j] = sIn[r][8 * blk + j];
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

    // epilogue: outputs (band, row) for this thread's column; every load is
    // issued before the first store (z(i) is written in place of z(i-2))
    double st[2] = {0.0, 0.0};
    bool bad = false;
    const int g1 = c01 + l1;
    const bool prox = a.mode == MODE_PROX;
    T zcr[JOINT ? PD_MAXC : 1][4], zpr[JOINT ? PD_MAXC : 1][4], wr[4];
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
        wr[o] = T(0);
        for (int cc = 0; cc < nch; ++cc) {
            zcr[cc][o] = T(0);
            zpr[cc][o] = T(0);
        }
        if (valid[o] && !toapx[o] && prox) {
            for (int cc = 0; cc < nch; ++cc) {
                const int64_t ci = (int64_t)(ch0 + cc) * p.plane + idxs[o];
                zcr[cc][o] = p.zc[ci];
                zpr[cc][o] = p.zp[ci];
            }
            if (p.wmap) wr[o] = p.wmap[(int64_t)ch0 * p.plane + idxs[o]];
        }
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int q = o >> 1, hx2 = o & 1;
        const int b = src + 2 * hx2;
        if (!valid[o]) continue;
        if (toapx[o]) {
            const int g2 = c02 + 2 * rblk + q;
            for (int cc = 0; cc < nch; ++cc)
                a.apx_out[(int64_t)(ch0 + cc) * a.apx_plane + (int64_t)g2 * M1c + g1] = res[cc][2 * q + hx2];
            continue;
        }
        const int64_t idx = idxs[o];
        if (!prox) {
            for (int cc = 0; cc < nch; ++cc) p.zn[(int64_t)(ch0 + cc) * p.plane + idx] = res[cc][2 * q + hx2];
            continue;
        }
        const int band = (b == 0) ? 0 : a.band_detail;
        if (!JOINT) {
            T w = p.wmap ? wr[o] : p.wlev[band];
            T y = zcr[0][o] + p.beta * (zcr[0][o] - zpr[0][o]);
            p.zn[(int64_t)ch0 * p.plane + idx] = prox1(y, res[0][2 * q + hx2], p.tau, w, st, bad);
        } else {
            T yv[PD_MAXC], vv[PD_MAXC];
            T nv = T(0);
            double ny = 0.0;
            for (int cc = 0; cc < nch; ++cc) {
                yv[cc] = zcr[cc][o] + p.beta * (zcr[cc][o] - zpr[cc][o]);
                vv[cc] = yv[cc] - p.tau * res[cc][2 * q + hx2];
                nv = fma(vv[cc], vv[cc], nv);
                ny += (double)yv[cc] * (double)yv[cc];
            }
            T w = p.wlev[band];
            T nrm = sqrt(nv);
            T sc = nrm > T(0) ? T(1) - p.tau * w / nrm : T(0);
            sc = sc > T(0) ? sc : T(0);
            bad |= !isfinite(nrm);
            st[0] += (double)w * sqrt(ny);
            for (int cc = 0; cc < nch; ++cc) {
                T z = vv[cc] * sc;
                p.zn[(int64_t)cc * p.plane + idx] = z;
                st[1] += ((double)z - (double)yv[cc]) * ((double)z - (double)yv[cc]);
            }
        }
    }
    if (a.mode == MODE_PROX) {
        if (p.slots) block_slot_add<2, NT>(st, p.slots + PD_NSLOT);
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
constexpr int CPT = 4;  // block elements per thread (64 x 64 / 1024)

// a mod M for a > -M*16 without integer division: a power-of-two M (mask =
// M-1, uniform per level) takes one AND; otherwise a few conditional steps.
__device__ __forceinline__ int wrapc(int a, int M, int mask)
{
    if (mask >= 0) return a & mask;
    while (a < 0) a += M;
    while (a >= M) a -= M;
    return a;
}
__device__ __forceinline__ int pmask(int M) { return (M & (M - 1)) == 0 ? M - 1 : -1; }

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

// Orders the LDS accesses of one wave: all lanes' writes before any later read.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Levels whose input holds at most this many values run on one wave with
// wave-level ordering only (no workgroup barriers on the critical path).
constexpr int WAVE_LEVEL_MAX = 256;

// One analysis level (rows then columns) over `nthr` threads (thread index
// `t`), M1 x M2 input in A -> Mallat bands in A, B as scratch.
template <typename T, bool WAVE>
__device__ __forceinline__ void ana_level(T *A, T *B, int pitch, int M1, int M2, const Filt<T> &f, int t,
                                          int nthr)
{
    const int h1 = M1 / 2, h2 = M2 / 2;
    const int k1 = pmask(M1), k2 = pmask(M2);
    for (int e = t; e < M2 * h1; e += nthr) {  // along x1
        int r, l;
        split(e, h1, r, l);
        const T *row = A + r * pitch;
        T x[22];  // inputs 2l-10 .. 2l+11
#pragma unroll
        for (int k = 0; k < 22; ++k) x[k] = row[wrapc(2 * l + k - 10, M1, k1)];
        T lo = T(0), hi = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            lo = fma(f.h[k], x[k + 10], lo);
            hi = fma(f.g[k], x[k], hi);
        }
        B[r * pitch + l] = lo;
        B[r * pitch + h1 + l] = hi;
    }
    if (WAVE) wave_sync();
    else __syncthreads();
    for (int e = t; e < h2 * M1; e += nthr) {  // along x2
        int l, c;
        split(e, M1, l, c);
        T x[22];
#pragma unroll
        for (int k = 0; k < 22; ++k) x[k] = B[wrapc(2 * l + k - 10, M2, k2) * pitch + c];
        T lo = T(0), hi = T(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            lo = fma(f.h[k], x[k + 10], lo);
            hi = fma(f.g[k], x[k], hi);
        }
        A[l * pitch + c] = lo;
        A[(h2 + l) * pitch + c] = hi;
    }
    if (WAVE) wave_sync();
    else __syncthreads();
}

// One synthesis level: coarse M1c x M2c bands in A -> 2 M1c x 2 M2c in A.
template <typename T, bool WAVE>
__device__ __forceinline__ void syn_level(T *A, T *B, int pitch, int M1c, int M2c, const Filt<T> &f, int t,
                                          int nthr)
{
    const int M1 = 2 * M1c, M2 = 2 * M2c;
    const int k1 = pmask(M1c), k2 = pmask(M2c);
    for (int e = t; e < M2c * M1; e += nthr) {  // along x2
        int pp, c;
        split(e, M1, pp, c);
        T lo[6], hi[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            lo[j] = A[wrapc(pp - 5 + j, M2c, k2) * pitch + c];
            hi[j] = A[(M2c + wrapc(pp + j, M2c, k2)) * pitch + c];
        }
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                acc = fma(f.h[par + 10 - 2 * j], lo[j], acc);
                acc = fma(f.g[par - 2 * j + 10], hi[j], acc);
            }
            B[(2 * pp + par) * pitch + c] = acc;
        }
    }
    if (WAVE) wave_sync();
    else __syncthreads();
    for (int e = t; e < M2 * M1c; e += nthr) {  // along x1
        int n, pp;
        split(e, M1c, n, pp);
        const T *row = B + n * pitch;
        T lo[6], hi[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            lo[j] = row[wrapc(pp - 5 + j, M1c, k1)];
            hi[j] = row[M1c + wrapc(pp + j, M1c, k1)];
        }
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                acc = fma(f.h[par + 10 - 2 * j], lo[j], acc);
                acc = fma(f.g[par - 2 * j + 10], hi[j], acc);
            }
            A[n * pitch + 2 * pp + par] = acc;
        }
    }
    if (WAVE) wave_sync();
    else __syncthreads();
}

// Analysis of all nlev levels of the block; the small ones on wave 0 alone.
// Ends with a workgroup barrier.
template <typename T>
__device__ void coarse_analysis(T *A, T *B, int pitch, int m1, int m2, int nlev, const Filt<T> &f)
{
    int M1 = m1, M2 = m2, lev = 0;
    for (; lev < nlev && M1 * M2 > WAVE_LEVEL_MAX; ++lev) {
        ana_level<T, false>(A, B, pitch, M1, M2, f, threadIdx.x, NTC);
        M1 /= 2;
        M2 /= 2;
    }
    if (lev < nlev) {
        if (threadIdx.x < 64) {
            for (; lev < nlev; ++lev) {
                ana_level<T, true>(A, B, pitch, M1, M2, f, threadIdx.x, 64);
                M1 /= 2;
                M2 /= 2;
            }
        }
        __syncthreads();
    }
}

// Synthesis of all nlev levels of the block (coarse to fine); the small ones
// on wave 0 alone.  Ends with a workgroup barrier.
template <typename T>
__device__ void coarse_synthesis(T *A, T *B, int pitch, int m1, int m2, int nlev, const Filt<T> &f)
{
    int lev = nlev - 1;
    if (threadIdx.x < 64) {
        for (; lev >= 0; --lev) {
            const int M1c = m1 >> (lev + 1), M2c = m2 >> (lev + 1);
            if (4 * M1c * M2c > WAVE_LEVEL_MAX) break;
            syn_level<T, true>(A, B, pitch, M1c, M2c, f, threadIdx.x, 64);
        }
    } else {
        for (; lev >= 0; --lev)
            if (4 * (m1 >> (lev + 1)) * (m2 >> (lev + 1)) > WAVE_LEVEL_MAX) break;
    }
    __syncthreads();
    for (; lev >= 0; --lev)
        syn_level<T, false>(A, B, pitch, m1 >> (lev + 1), m2 >> (lev + 1), f, threadIdx.x, NTC);
}

template <typename T>
__device__ __forceinline__ void coarse_body(const CoarseArgs<T> &a, int bz)
{
    extern __shared__ unsigned char lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    const ProxArgs<T> &p = a.p;
    const int m1 = a.m1, m2 = a.m2, pitch = m1 + 1;
    const int nch = p.joint ? p.C : 1;
    const int ch0 = p.joint ? 0 : bz;
    T *B = lds + (size_t)nch * m2 * pitch;
    const int cnt = m1 * m2;  // <= CPT * NTC
    const int tid = threadIdx.x;
    const bool ana = (a.ops & COARSE_ANA) != 0, prox = (a.ops & COARSE_PROX) != 0;

    // 1. all global loads: analysis input (or y for synthesis only), and the
    //    state/weights the prox needs, for this thread's block elements
    T zcr[PD_MAXC][CPT], zpr[PD_MAXC][CPT], wr[CPT];
    for (int cc = 0; cc < nch; ++cc) {
        T *A = lds + (size_t)cc * m2 * pitch;
        const int64_t ch = ch0 + cc;
        T v[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int e = tid + k * NTC;
            v[k] = T(0);
            zcr[cc][k] = T(0);
            zpr[cc][k] = T(0);
            if (e < cnt) {
                const int r = e / m1, c = e - r * m1;
                const int64_t idx = ch * p.plane + (int64_t)r * p.pitch + c;
                if (ana) v[k] = a.apx_in[ch * a.apx_in_plane + e];
                if (!ana || prox) {
                    zcr[cc][k] = p.zc[idx];
                    zpr[cc][k] = p.zp[idx];
                }
                if (cc == 0) wr[k] = (prox && p.wmap) ? p.wmap[idx] : T(0);
            }
        }
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int e = tid + k * NTC;
            if (e < cnt) {
                const int r = e / m1, c = e - r * m1;
                A[r * pitch + c] = ana ? v[k] : zcr[cc][k] + p.beta * (zcr[cc][k] - zpr[cc][k]);
            }
        }
    }
    __syncthreads();

    if (ana) {
        for (int cc = 0; cc < nch; ++cc)
            coarse_analysis<T>(lds + (size_t)cc * m2 * pitch, B, pitch, m1, m2, a.nlev, a.f);
        if (!prox) {  // plain forward transform
            for (int cc = 0; cc < nch; ++cc) {
                const T *A = lds + (size_t)cc * m2 * pitch;
                for (int e = tid; e < cnt; e += NTC) {
                    int r = e / m1, c = e - r * m1;
                    p.zn[(int64_t)(ch0 + cc) * p.plane + (int64_t)r * p.pitch + c] = A[r * pitch + c];
                }
            }
            return;
        }
        // 2. gradient step + prox + momentum on the coarse block
        double st[2] = {0.0, 0.0};
        bool bad = false;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int e = tid + k * NTC;
            if (e >= cnt) continue;
            const int r = e / m1, c = e - r * m1;
            // band index: finest level of the block whose detail region holds (r, c)
            int band = 0;
            for (int lev = 0; lev < a.nlev; ++lev)
                if (r >= (m2 >> (lev + 1)) || c >= (m1 >> (lev + 1))) {
                    band = a.band_top - lev;
                    break;
                }
            const int64_t idx = (int64_t)r * p.pitch + c;
            if (!p.joint) {
                T *A = lds;
                T w = p.wmap ? wr[k] : p.wlev[band];
                T y = zcr[0][k] + p.beta * (zcr[0][k] - zpr[0][k]);
                T z = prox1(y, A[r * pitch + c], p.tau, w, st, bad);
                p.zn[(int64_t)ch0 * p.plane + idx] = z;
                A[r * pitch + c] = z + a.beta_next * (z - zcr[0][k]);
            } else {
                T yv[PD_MAXC], vv[PD_MAXC];
                T nv = T(0);
                double ny = 0.0;
                for (int cc = 0; cc < nch; ++cc) {
                    yv[cc] = zcr[cc][k] + p.beta * (zcr[cc][k] - zpr[cc][k]);
                    vv[cc] = yv[cc] - p.tau * lds[(size_t)cc * m2 * pitch + r * pitch + c];
                    nv = fma(vv[cc], vv[cc], nv);
                    ny += (double)yv[cc] * (double)yv[cc];
                }
                T w = p.wlev[band];
                T nrm = sqrt(nv);
                T sc = nrm > T(0) ? T(1) - p.tau * w / nrm : T(0);
                sc = sc > T(0) ? sc : T(0);
                bad |= !isfinite(nrm);
                st[0] += (double)w * sqrt(ny);
                for (int cc = 0; cc < nch; ++cc) {
                    T z = vv[cc] * sc;
                    p.zn[(int64_t)cc * p.plane + idx] = z;
                    st[1] += ((double)z - (double)yv[cc]) * ((double)z - (double)yv[cc]);
                    lds[(size_t)cc * m2 * pitch + r * pitch + c] = z + a.beta_next * (z - zcr[cc][k]);
                }
            }
        }
        if (bad) atomicOr(p.flag, 1);
        if (p.slots) block_slot_add<2, NTC>(st, p.slots + PD_NSLOT);  // contains a barrier
        else __syncthreads();
    }
    if (!(a.ops & COARSE_SYN)) return;
    // 3. synthesis of the block back to the level lc-1 approximation
    for (int cc = 0; cc < nch; ++cc) {
        T *A = lds + (size_t)cc * m2 * pitch;
        coarse_synthesis<T>(A, B, pitch, m1, m2, a.nlev, a.f);
        for (int e = tid; e < cnt; e += NTC) {
            int r = e / m1, c = e - r * m1;
            a.apx_out[(int64_t)(ch0 + cc) * a.apx_out_plane + e] = A[r * pitch + c];
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

__global__ __launch_bounds__(256) void k_stats_finalize_b(double *const *__restrict__ ring,
                                                           double *const *__restrict__ stats, int it0)
{
    const int it = it0 + blockIdx.x, img = blockIdx.y;
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
// A workgroup produces a 32-row x 46-column tile of s, so the column passes
// work on exactly 64 columns: one wave64 per block of rows with lane = column,
// which makes the row profiles wave-uniform (scalar loads).  Profiles narrower
// than RM = 9 are zero-padded.
// ===========================================================================
constexpr int RM = PD_MAX_RADIUS;
constexpr int BW = 64;                 // columns of t, r, u
constexpr int BT1 = BW - 2 * RM;       // 46 output columns
constexpr int BT2 = 32;                // output rows
constexpr int BX1 = BT1 + 4 * RM;      // 82 x columns
constexpr int BX2 = BT2 + 4 * RM;      // 68 x / t rows
constexpr int BR2 = BT2 + 2 * RM;      // 50 r rows
constexpr int XP = 84;                 // LDS pitch of x (multiple of 4)
constexpr int TP = 68;                 // LDS pitch of t, r, u (multiple of 4)
static_assert(BX2 % (NT / 64) == 0 && BX1 <= 128 && BX1 > 64, "blur load rows/columns");
constexpr int RVH = 5;                 // rows per column task in the r pass (50 = 10 x 5)
constexpr int UVH = 4;                 // rows per column task in the u pass (32 = 8 x 4)

template <typename T>
__device__ __forceinline__ void blur_body(const BlurArgs<T> &a, int bx, int by, int bz)
{
    __shared__ T sA[BX2 * XP];           // x, later r (BR2 x TP)
    __shared__ T sB[BX2 * TP];           // t, later u (BT2 x TP)
    __shared__ T sK[BX2][2 * RM + 2];    // profiles of the rows of x / t
    const int n1 = a.n1, n2 = a.n2, R = a.R, W = 2 * R + 1;
    const int64_t ch = bz;
    const int o1 = bx * BT1, o2 = by * BT2;
    const T *x = a.x + ch * a.plane;
    const T *f0 = a.f0 ? a.f0 + ch * a.plane : nullptr;
    const T *__restrict__ taps = a.taps;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);

    {
        // load: lane = column (two chunks: 64 + 18), wave = rows (17 each)
        constexpr int RPW = BX2 / (NT / 64);
        const int qa = wrap(o1 - 2 * RM + lane, n1);
        const bool okb = 64 + lane < BX1;
        const int qb = okb ? wrap(o1 - 2 * RM + 64 + lane, n1) : 0;
        T va[RPW], vb[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + i * (NT / 64);
            const T *rowp = x + (int64_t)wrap(o2 - 2 * RM + r, n2) * n1;
            va[i] = rowp[qa];
            vb[i] = okb ? rowp[qb] : T(0);
        }
        for (int e = tid; e < BX2 * (2 * RM + 1); e += NT) {
            int r = e / (2 * RM + 1), d = e - r * (2 * RM + 1) - RM;
            int row = wrap(o2 - 2 * RM + r, n2);
            sK[r][d + RM] = (d >= -R && d <= R) ? taps[(int64_t)row * W + d + R] : T(0);
        }
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int r = wv + i * (NT / 64);
            sA[r * XP + lane] = va[i];
            if (okb) sA[r * XP + 64 + lane] = vb[i];
        }
    }
    __syncthreads();

    // t: rows [0, BX2) (pixel row o2-2RM+r), columns [0, BW) (pixel col o1-RM+c)
    for (int t = tid; t < BX2 * (BW / 4); t += NT) {
        int r = t / (BW / 4), blk = t - r * (BW / 4);
        T xv[4 + 2 * RM];
#pragma unroll
        for (int j = 0; j < 4 + 2 * RM; ++j) xv[j] = sA[r * XP + 4 * blk + j];
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
    __syncthreads();

    // r: rows [0, BR2) (pixel row o2-RM+r), lane = column; the source t row of
    // output row r0+k and offset m is r0+m with profile index k+2RM-m.
    double st[1] = {0.0};
    for (int blk = wv; blk < BR2 / RVH; blk += NT / 64) {
        const int r0 = blk * RVH;
        T acc[RVH];
        T f0v[RVH];
        const int q1 = wrap(o1 - RM + lane, n1);
#pragma unroll
        for (int k = 0; k < RVH; ++k) {
            acc[k] = T(0);
            f0v[k] = a.f0 ? f0[(int64_t)wrap(o2 - RM + r0 + k, n2) * n1 + q1] : T(0);
        }
#pragma unroll
        for (int m = 0; m < RVH + 2 * RM; ++m) {
            const T tv = sB[(r0 + m) * TP + lane];
            const T *kr = &sK[r0 + m][RM];  // profile of source row r0+m (broadcast reads)
#pragma unroll
            for (int k = 0; k < RVH; ++k) {
                const int d = k + RM - m;  // displacement x2 - y2
                if (d >= -RM && d <= RM) acc[k] = fma(kr[d], tv, acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < RVH; ++k) {
            T rv = acc[k] - f0v[k];
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
    for (int blk = wv; blk < BT2 / UVH; blk += NT / 64) {
        const int q0 = blk * UVH;
        T rv[UVH + 2 * RM];
#pragma unroll
        for (int j = 0; j < UVH + 2 * RM; ++j) rv[j] = sA[(q0 + j) * TP + lane];
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
    for (int t = tid; t < BT2 * ((BT1 + 3) / 4); t += NT) {
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
    if (a.slots) block_slot_add<1, NT>(st, a.slots);
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
        if (wbar && act) wbar[e] -= tau * zb * (zv > T(0) ? T(1) : T(-1));
    }
}

// ybar = vbar - tau gbar; with b = b_{i-1}:  zbar <- zbarm + (1+b) ybar,
// zbarm <- -b ybar  (i >= 2); for i = 1 zbar <- ybar + zbarm (the init's adjoint).
template <typename T>
__global__ void k_rev_combine(const T *vbar, const T *gbar, T *zbar, T *zbarm, T tau, T b, int first, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const T yb = vbar[e] - tau * gbar[e];
        if (first) {
            zbar[e] = yb + zbarm[e];
        } else {
            zbar[e] = zbarm[e] + (T(1) + b) * yb;
            zbarm[e] = -b * yb;
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

template <typename T>
__global__ __launch_bounds__(NT) void k_synth(SynthArgs<T> a) { synth_body<T>(a, blockIdx.x, blockIdx.y, blockIdx.z); }

template <typename T, bool JOINT>
__global__ __launch_bounds__(NT) void k_analysis(AnalysisArgs<T> a)
{
    analysis_body<T, JOINT>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T>
__global__ __launch_bounds__(NTC) void k_coarse(CoarseArgs<T> a) { coarse_body<T>(a, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(NT) void k_blur(BlurArgs<T> a) { blur_body<T>(a, blockIdx.x, blockIdx.y, blockIdx.z); }

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

template <typename T>
__device__ __forceinline__ void apply_dyn(ProxArgs<T> &p, const Dyn<T> &d)
{
    if (d.parity) {
        const T *t = p.zc;
        p.zc = p.zp;
        p.zp = t;
    }
    p.zn = const_cast<T *>(p.zp);  // z(i) is written in place of z(i-2)
    p.beta = d.beta;
    if (p.slots) p.slots += (size_t)d.ring * 3 * PD_NSLOT;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_synth_b(const SynthArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                 int n, Dyn<T> d)
{
    const int img = locate(start, n, blockIdx.x);
    SynthArgs<T> a = tab[img];
    if (d.parity) {
        const T *t = a.zc;
        a.zc = a.zp;
        a.zp = t;
    }
    a.beta = d.beta;
    int loc = blockIdx.x - start[img];
    const int bx = loc % a.tx;
    loc /= a.tx;
    synth_body<T>(a, bx, loc % a.ty, loc / a.ty);
}

template <typename T, bool JOINT>
__global__ __launch_bounds__(NT) void k_analysis_b(const AnalysisArgs<T> *__restrict__ tab,
                                                    const int *__restrict__ start, int n, Dyn<T> d)
{
    const int img = locate(start, n, blockIdx.x);
    AnalysisArgs<T> a = tab[img];
    if (a.mode == MODE_PROX) apply_dyn<T>(a.p, d);
    int loc = blockIdx.x - start[img];
    const int bx = loc % a.tx;
    loc /= a.tx;
    analysis_body<T, JOINT>(a, bx, loc % a.ty, loc / a.ty);
}

template <typename T>
__global__ __launch_bounds__(NTC) void k_coarse_b(const CoarseArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                   int n, Dyn<T> d)
{
    const int img = locate(start, n, blockIdx.x);
    CoarseArgs<T> a = tab[img];
    if (a.ops & COARSE_PROX) {
        apply_dyn<T>(a.p, d);
        a.beta_next = d.beta_next;
    } else if (!(a.ops & COARSE_ANA)) {  // synthesis only: y from the state
        if (d.parity) {
            const T *t = a.p.zc;
            a.p.zc = a.p.zp;
            a.p.zp = t;
        }
        a.p.beta = d.beta;
    }
    coarse_body<T>(a, blockIdx.x - start[img]);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_blur_b(const BlurArgs<T> *__restrict__ tab, const int *__restrict__ start,
                                                int n, int ring)
{
    const int img = locate(start, n, blockIdx.x);
    BlurArgs<T> a = tab[img];
    if (a.slots) a.slots += (size_t)ring * 3 * PD_NSLOT;
    int loc = blockIdx.x - start[img];
    const int bx = loc % a.tx;
    loc /= a.tx;
    blur_body<T>(a, bx, loc % a.ty, loc / a.ty);
}

// ------------------------------------------------------------ launchers ---
template <typename T>
hipError_t launch_synth(const SynthArgs<T> &a, int C, hipStream_t s)
{
    dim3 grid((a.M1c + SP - 1) / SP, (a.M2c + SP - 1) / SP, C);
    hipLaunchKernelGGL(k_synth<T>, grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_analysis(const AnalysisArgs<T> &a, hipStream_t s)
{
    dim3 grid((a.M1c + TC - 1) / TC, (a.M2c + TC - 1) / TC, a.p.joint ? 1 : a.p.C);
    if (a.p.joint)
        hipLaunchKernelGGL((k_analysis<T, true>), grid, dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_analysis<T, false>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename T>
size_t coarse_lds_bytes(int m1, int m2, int chans)
{
    return sizeof(T) * (size_t)(chans + 1) * m2 * (m1 + 1);
}

template <typename T>
hipError_t launch_coarse(const CoarseArgs<T> &a, int groups, hipStream_t s)
{
    const int chans = a.p.joint ? a.p.C : 1;
    size_t lds = coarse_lds_bytes<T>(a.m1, a.m2, chans);
    hipLaunchKernelGGL(k_coarse<T>, dim3(groups), dim3(NTC), lds, s, a);
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

template <typename T>
hipError_t launch_synth_b(const SynthArgs<T> *tab, const int *start, int n, int tiles, Dyn<T> d, hipStream_t s)
{
    hipLaunchKernelGGL(k_synth_b<T>, dim3(tiles), dim3(NT), 0, s, tab, start, n, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_analysis_b(const AnalysisArgs<T> *tab, const int *start, int n, int tiles, bool joint, Dyn<T> d,
                             hipStream_t s)
{
    if (joint)
        hipLaunchKernelGGL((k_analysis_b<T, true>), dim3(tiles), dim3(NT), 0, s, tab, start, n, d);
    else
        hipLaunchKernelGGL((k_analysis_b<T, false>), dim3(tiles), dim3(NT), 0, s, tab, start, n, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_b(const CoarseArgs<T> *tab, const int *start, int n, int groups, size_t lds, Dyn<T> d,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_coarse_b<T>, dim3(groups), dim3(NTC), lds, s, tab, start, n, d);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_blur_b(const BlurArgs<T> *tab, const int *start, int n, int tiles, int ring, hipStream_t s)
{
    hipLaunchKernelGGL(k_blur_b<T>, dim3(tiles), dim3(NT), 0, s, tab, start, n, ring);
    return hipGetLastError();
}

hipError_t launch_stats_finalize_b(double *const *ring, double *const *stats, int n, int it0, int count,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_finalize_b, dim3(count, n), dim3(256), 0, s, ring, stats, it0);
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
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_rev_combine<T>, dim3(ew_blocks(n)), dim3(256), 0, s, vbar, gbar, zbar, zbarm, tau, b, first, n);
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
    template hipError_t launch_rev_combine<T>(const T *, const T *, T *, T *, T, T, int, int64_t,       \
                                              hipStream_t);                                             \
    template hipError_t launch_add<T>(const T *, T *, int64_t, hipStream_t);                            \
    template hipError_t launch_expand_weights<T>(T *, const T *, int, int, int, int, hipStream_t);
PD_INST_REV(float)
PD_INST_REV(double)

void tiles_synth(int M1c, int M2c, int *tx, int *ty) { *tx = (M1c + SP - 1) / SP; *ty = (M2c + SP - 1) / SP; }
void tiles_analysis(int M1c, int M2c, int *tx, int *ty) { *tx = (M1c + TC - 1) / TC; *ty = (M2c + TC - 1) / TC; }
void tiles_blur(int n1, int n2, int *tx, int *ty) { *tx = (n1 + BT1 - 1) / BT1; *ty = (n2 + BT2 - 1) / BT2; }

hipError_t launch_stats_finalize(double *ring, double *stats, int it0, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_stats_finalize, dim3(count), dim3(256), 0, s, ring, stats, it0);
    return hipGetLastError();
}

#define PD_INST(T)                                                                          \
    template hipError_t launch_synth<T>(const SynthArgs<T> &, int, hipStream_t);           \
    template hipError_t launch_analysis<T>(const AnalysisArgs<T> &, hipStream_t);          \
    template hipError_t launch_coarse<T>(const CoarseArgs<T> &, int, hipStream_t);         \
    template size_t coarse_lds_bytes<T>(int, int, int);                                    \
    template hipError_t launch_blur<T>(const BlurArgs<T> &, bool, hipStream_t);            \
    template hipError_t launch_blur_single<T>(const BlurArgs<T> &, int, hipStream_t);      \
    template hipError_t launch_copy<T>(const T *, T *, int64_t, hipStream_t);                   \
    template hipError_t launch_synth_b<T>(const SynthArgs<T> *, const int *, int, int, Dyn<T>, hipStream_t); \
    template hipError_t launch_analysis_b<T>(const AnalysisArgs<T> *, const int *, int, int, bool, Dyn<T>,     \
                                             hipStream_t);                                                      \
    template hipError_t launch_coarse_b<T>(const CoarseArgs<T> *, const int *, int, int, size_t, Dyn<T>,       \
                                           hipStream_t);                                                        \
    template hipError_t launch_blur_b<T>(const BlurArgs<T> *, const int *, int, int, int, hipStream_t);
PD_INST(float)
PD_INST(double)

}  // namespace pd
