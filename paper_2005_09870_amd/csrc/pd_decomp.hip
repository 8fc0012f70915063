// pd_decomp.hip -- gfx950 kernels of Algorithm 1 (Section 3.2; Section 5),
// FP64.
//
// The sub-bands of A_k = Psi^* U_k Psi are circulant (Section 5.1), so A~_k is
// held as the kept entries of its generators: for a source band b' and a
// finer-or-equal target band b, the column of a source at band position l'
// is the generator column shifted by 2^(lev_b' - lev_b) l' in b's grid; for a
// coarser target, the row of a target at l is the generator row shifted by
// 2^(lev_b - lev_b') l in b''s grid.  C_k = A~_k B_k is formed column by column:
// every nonzero of a column of B_k spreads its generator entries into a dense
// FP64 accumulator of that column held in LDS (one workgroup per column and
// 16384-row part), which is then added to the column and compacted in row order.
#include <hip/hip_runtime.h>

#include "pd_decomp.h"

namespace pd {

namespace {

constexpr int NTD = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + NTD - 1) / NTD); }

__global__ void k_dec_dirac(double *planes, int64_t base, int64_t N)
{
    const int p = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * NTD + threadIdx.x; i < N; i += (int64_t)gridDim.x * NTD)
        planes[(int64_t)p * N + i] = i == base + p ? 1.0 : 0.0;
}

__global__ void k_dec_dirac_at(double *planes, const int *pos, int64_t N)
{
    const int p = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * NTD + threadIdx.x; i < N; i += (int64_t)gridDim.x * NTD)
        planes[(int64_t)p * N + i] = i == pos[p] ? 1.0 : 0.0;
}

__global__ void k_dec_conv(const double *in, double *out, const double *u, int R, int n1, int n2, int transpose)
{
    const int64_t N = (int64_t)n1 * n2;
    const int64_t i = (int64_t)blockIdx.x * NTD + threadIdx.x;
    if (i >= N) return;
    const double *x = in + (int64_t)blockIdx.y * N;
    const int i2 = (int)(i / n1), i1 = (int)(i - (int64_t)i2 * n1);
    const int W = 2 * R + 1;
    const int sg = transpose ? 1 : -1;  // convolution reads x(p - d), the correlation x(p + d)
    double acc = 0.0;
    for (int d2 = -R; d2 <= R; ++d2) {
        const int r = (((i2 + sg * d2) % n2) + n2) % n2;
        for (int d1 = -R; d1 <= R; ++d1) {
            const int c = (((i1 + sg * d1) % n1) + n1) % n1;
            acc = fma(u[(d2 + R) * W + d1 + R], x[(int64_t)r * n1 + c], acc);
        }
    }
    out[(int64_t)blockIdx.y * N + i] = acc;
}

__global__ void k_dec_mul(const double *in, const double *v, double *out, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * NTD + threadIdx.x;
    if (i >= N) return;
    const int64_t o = (int64_t)blockIdx.y * N + i;
    out[o] = v[i] * in[o];
}

// band index of Mallat position (i2, i1): levels 1..L with orientations 1..3, then the approximation
__device__ __forceinline__ int band_index(int i2, int i1, int n1, int n2, int nb)
{
    const int L = (nb - 1) / 3;
    for (int lev = 1; lev <= L; ++lev) {
        const int h2 = n2 >> lev, h1 = n1 >> lev;
        if (i2 >= h2 || i1 >= h1) return (lev - 1) * 3 + (i2 < h2 ? 0 : (i1 < h1 ? 1 : 2));
    }
    return nb - 1;
}

// Accumulator of one part of a column in LDS: 16384 FP64 values (128 KiB of the CU's 160 KiB);
// part p of the grid covers Mallat positions [p DEC_LDS, (p + 1) DEC_LDS).
constexpr int DEC_LDS = 16384;
constexpr int NTA = 512;

__global__ __launch_bounds__(NTA) void k_dec_acc(const double *y, double *acc, DecTables t, int k)
{
    __shared__ double part[DEC_LDS];
    const int64_t N = (int64_t)t.n1 * t.n2;
    const int64_t p0 = (int64_t)blockIdx.y * DEC_LDS;
    const int64_t plen = N - p0 < DEC_LDS ? N - p0 : DEC_LDS;
    for (int i = threadIdx.x; i < DEC_LDS; i += NTA) part[i] = 0.0;
    __syncthreads();
    const double *yc = y + (int64_t)blockIdx.x * N;
    for (int64_t nu = threadIdx.x; nu < N; nu += NTA) {
        const double yv = yc[nu];
        if (yv == 0.0) continue;
        const int i2 = (int)(nu / t.n1), i1 = (int)(nu - (int64_t)i2 * t.n1);
        const int bs = band_index(i2, i1, t.n1, t.n2, t.nb);
        const DecBand S = t.bands[bs];
        const int l2 = i2 - S.o2, l1 = i1 - S.o1;
        for (int b = 0; b < t.nb; ++b) {
            const DecBand B = t.bands[b];
            // skip a target band whose rows lie outside this part
            const int64_t first = (int64_t)B.o2 * t.n1, last = (int64_t)(B.o2 + B.g2) * t.n1;
            if (last <= p0 || first >= p0 + plen) continue;
            const int64_t p = ((int64_t)k * t.nb + bs) * t.nb + b;
            const DecEntry *e = t.ent + t.off[p];
            if (B.lev <= S.lev) {  // finer-or-equal target: the generator column shifted by f l'
                const int f = 1 << (S.lev - B.lev);
                const int c = t.cnt[p];
                for (int q = 0; q < c; ++q) {
                    const DecEntry en = e[q];
                    const int r2 = (en.q2 + f * l2) % B.g2, r1 = (en.q1 + f * l1) % B.g1;
                    const int64_t ti = (int64_t)(B.o2 + r2) * t.n1 + B.o1 + r1 - p0;
                    if (ti >= 0 && ti < plen) atomicAdd(part + ti, yv * en.val);
                }
            } else {  // coarser target: the generator rows whose shift lands on l'
                const int f = 1 << (B.lev - S.lev);
                const int r = (l2 % f) * f + (l1 % f);
                const int *rs = t.res + t.roff[p];
                for (int q = rs[r]; q < rs[r + 1]; ++q) {
                    const DecEntry en = e[q];
                    const int r2 = ((((l2 - en.q2) / f) % B.g2) + B.g2) % B.g2;
                    const int r1 = ((((l1 - en.q1) / f) % B.g1) + B.g1) % B.g1;
                    const int64_t ti = (int64_t)(B.o2 + r2) * t.n1 + B.o1 + r1 - p0;
                    if (ti >= 0 && ti < plen) atomicAdd(part + ti, yv * en.val);
                }
            }
        }
    }
    __syncthreads();
    double *ac = acc + (int64_t)blockIdx.x * N + p0;
    for (int i = threadIdx.x; i < plen; i += NTA) ac[i] += part[i];
}

__global__ __launch_bounds__(NTD) void k_dec_count(const double *acc, int64_t N, int64_t *cnt)
{
    __shared__ int red[NTD / 64];
    const double *ac = acc + (int64_t)blockIdx.x * N;
    int c = 0;
    for (int64_t i = threadIdx.x; i < N; i += NTD) c += ac[i] != 0.0;
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int w = 0; w < NTD / 64; ++w) s += red[w];
        cnt[blockIdx.x] = s;
    }
}

// ordered compaction: chunks of NTD entries, wave ballots and an LDS prefix over the waves
__global__ __launch_bounds__(NTD) void k_dec_fill(const double *acc, int64_t N, const int64_t *base, int *rows,
                                                  double *vals)
{
    __shared__ int wsum[NTD / 64];
    const double *ac = acc + (int64_t)blockIdx.x * N;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t pos = base[blockIdx.x];
    for (int64_t c0 = 0; c0 < N; c0 += NTD) {
        const int64_t i = c0 + threadIdx.x;
        const double v = i < N ? ac[i] : 0.0;
        const bool nz = v != 0.0;
        const unsigned long long bal = __ballot(nz);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < NTD / 64; ++w) {
            off += w < wv ? wsum[w] : 0;
            tot += wsum[w];
        }
        if (nz) {
            rows[pos + off + before] = (int)i;
            vals[pos + off + before] = v;
        }
        pos += tot;
        __syncthreads();  // wsum is rewritten by the next chunk
    }
}

}  // namespace

hipError_t launch_dec_dirac(double *planes, int64_t base, int P, int64_t N, hipStream_t s)
{
    unsigned g = nblk(N);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_dec_dirac, dim3(g, P), dim3(NTD), 0, s, planes, base, N);
    return hipGetLastError();
}

hipError_t launch_dec_dirac_at(double *planes, const int *pos, int P, int64_t N, hipStream_t s)
{
    unsigned g = nblk(N);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_dec_dirac_at, dim3(g, P), dim3(NTD), 0, s, planes, pos, N);
    return hipGetLastError();
}

hipError_t launch_dec_conv(const double *in, double *out, int P, const double *u, int R, int n1, int n2,
                           int transpose, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_conv, dim3(nblk((int64_t)n1 * n2), P), dim3(NTD), 0, s, in, out, u, R, n1, n2,
                       transpose);
    return hipGetLastError();
}

hipError_t launch_dec_mul(const double *in, const double *v, double *out, int P, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_mul, dim3(nblk(N), P), dim3(NTD), 0, s, in, v, out, N);
    return hipGetLastError();
}

hipError_t launch_dec_acc(const double *y, double *acc, int P, const DecTables &t, int k, hipStream_t s)
{
    const int64_t N = (int64_t)t.n1 * t.n2;
    const unsigned parts = (unsigned)((N + DEC_LDS - 1) / DEC_LDS);
    hipLaunchKernelGGL(k_dec_acc, dim3(P, parts), dim3(NTA), 0, s, y, acc, t, k);
    return hipGetLastError();
}

hipError_t launch_dec_count(const double *acc, int P, int64_t N, int64_t *cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_count, dim3(P), dim3(NTD), 0, s, acc, N, cnt);
    return hipGetLastError();
}

hipError_t launch_dec_fill(const double *acc, int P, int64_t N, const int64_t *base, int *rows, double *vals,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_dec_fill, dim3(P), dim3(NTD), 0, s, acc, N, base, rows, vals);
    return hipGetLastError();
}

}  // namespace pd
