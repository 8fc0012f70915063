// pd_kernels.h -- argument blocks and launchers of the gfx950 kernels
// (internal to libpd; the public interface is include/pd.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#define PD_MAXC 4
#define PD_MAXL 16
#define PD_MAX_RADIUS 9
#define PD_NSLOT 64   // partial-sum slots per statistic (spreads FP64 atomics)
#define PD_RING 64    // iterations whose partial sums are kept before a finalise
#define PD_TAIL_MAX 64 // coarse levels whose input has at most this many values are one matrix apply

namespace pd {

// Filter bank zero-padded to 12 taps: h[k], k = 0..11, and g[k + 10] for
// k = -10..1 with g[k] = (-1)^(1-k) h[1-k] (Section 2.1).
template <typename T>
struct Filt {
    T h[12];
    T g[12];
};

// One synthesis level: coarse size M1c x M2c -> fine 2*M1c x 2*M2c.
// Coefficients y = zc + beta (zc - zp) (row pitch `pitch`, plane stride
// `plane`); the approximation band comes from `apx` (dense M2c x M1c per
// channel, stride apx_plane) or, if apx == nullptr, from the coefficient
// state at [0,M2c) x [0,M1c).
// Iteration number read from device memory when a launch sits in a replayed
// graph: i = *it_dev + it_off (it_dev == nullptr: the by-value momenta apply).
struct DevIter {
    const int *it_dev;
    int it_off;
};

template <typename T>
struct SynthArgs {
    Filt<T> f;
    const T *zc, *zp;
    T beta;
    DevIter di;
    int64_t plane;
    int pitch;
    const T *apx;
    int64_t apx_plane;
    T *out;
    int out_pitch;
    int64_t out_plane;
    int M1c, M2c;
    int tx, ty;             // tiles along x1, x2 (batched launches)
};

enum { MODE_PLAIN = 0, MODE_PROX = 1 };

// Prox / weight parameters shared by the analysis and coarse kernels.
template <typename T>
struct ProxArgs {
    const T *zc, *zp;
    T *zn;
    T *zsave;               // nullptr, or a second plane that also receives z(i) (the
                            // recomputation's per-iteration record in pd_backward)
    T beta, tau;
    int64_t plane;
    int pitch;
    const T *wmap;          // per-coefficient weights or nullptr
    T wlev[PD_MAXL + 1];    // per-band weights
    int joint, C;
    double *slots;          // this iteration's [3][PD_NSLOT] partial sums (nullptr: no
                            // statistics): 1/2||r||^2, sum w|y|, sum (z-y)^2
    int *flag;              // set to 1 if a prox argument is not finite
    DevIter di;             // beta (and the coarse kernel's beta_next) from the device iteration
};

// One analysis level: fine input 2*M1c x 2*M2c -> four coarse M1c x M2c
// bands.  MODE_PLAIN stores the detail bands (and, if last, the approximation
// band) in zn.  MODE_PROX treats them as the gradient g and stores
// z = Prox(y - tau g) in zn with y = zc + beta (zc - zp).  If !last the
// approximation band goes to apx_out (dense, stride apx_plane).
template <typename T>
struct AnalysisArgs {
    Filt<T> f;
    const T *in;
    int in_pitch;
    int64_t in_plane;
    int M1c, M2c;
    int last;
    T *apx_out;
    int64_t apx_plane;
    int mode;
    int band_detail;        // band index k of this level's detail bands
    int tx, ty;             // tiles along x1, x2 (batched launches)
    ProxArgs<T> p;
};

// All levels lc..L in one workgroup per channel (per image in joint mode):
// the approximation of level lc-1 (m1 x m2, dense) is analysed, the prox and
// momentum are applied to the coarse block [0,m2) x [0,m1) of the Mallat
// plane, and/or the block is synthesised back to a level lc-1 approximation.
enum { COARSE_ANA = 1, COARSE_PROX = 2, COARSE_SYN = 4, COARSE_REVCM = 8 };
template <typename T>
struct CoarseArgs {
    Filt<T> f;
    int ops;                // COARSE_* bits
    int m1, m2;             // size of the level lc-1 approximation
    int nlev;               // number of levels in the block (L - lc + 1)
    int band_top;           // band index k of the finest level in the block (L+1-lc)
    const T *apx_in;        // analysis input (dense m2 x m1 per channel)
    int64_t apx_in_plane;
    T *apx_out;             // synthesis output (dense m2 x m1 per channel)
    int64_t apx_out_plane;
    T beta_next;            // momentum of the next iteration's y (COARSE_PROX|COARSE_SYN)
    int kw;                 // levels of the block done level by level (input > PD_TAIL_MAX values)
    int tM1, tM2;           // input size of the remaining levels (the tail), tM1*tM2 <= PD_TAIL_MAX
    const T *tail;          // [2][tn][tn], tn = tM1*tM2: the tail's analysis matrix (row = output,
                            // Mallat position) then its transpose (synthesis); nullptr if kw == nlev
    ProxArgs<T> p;          // in PLAIN analysis (ops == ANA) zn receives coefficients
    // Reverse sweep (COARSE_REVCM, one channel per workgroup): after the analysis
    // of gbar, the combine of iteration i and the mask of iteration i-1 on the
    // block (vbar in p.zc, z(i-1) in p.zp, tau in p.tau; b = b_{i-1}), then the
    // synthesis of the new vbar (with COARSE_SYN)
    T *rv_vbar = nullptr, *rv_zbar = nullptr, *rv_zbarm = nullptr, *rv_wbar = nullptr;
    T rv_b = T(0);
    int rv_first = 0;
    DevIter rv_di{nullptr, 0};
};

// The joint prox on a coarse block (m1 x m2 at the top left of each channel's
// Mallat plane) from the coefficients g that a per-channel coarse analysis
// wrote at their Mallat positions of a scratch plane.
template <typename T>
struct JProxArgs {
    const T *g;             // [C][n2][n1] coefficients of the transformed gradient (read in the region)
    int m1, m2, nlev, band_top;  // region = top-left m2 x m1 of the Mallat plane, its levels,
                                 // band index of its finest detail level
    ProxArgs<T> p;          // zc, zp, zn, beta, tau, weights, slots, flag, di
};

// Fused r = H x - f0, s = H^T r (or a single pass for the building block).
template <typename T>
struct BlurArgs {
    const T *x, *f0;
    T *s;
    const T *taps;
    int n1, n2, C, R;
    int64_t plane;
    double *slots;          // [3][PD_NSLOT] partial sums; 1/2 ||r||^2 goes to row 0
    int tx, ty;             // tiles along x1, x2 (batched launches)
    T *racc;                // reverse mode: racc += rscale * r (nullptr: off); f0 may be nullptr
    T rscale;
    T *r;                   // plane for r = Hx - f0 of the two-kernel variant (nullptr: fused only)
    const T *tabs;          // [2][n2][2 PD_MAX_RADIUS + 2] profile tables of that variant
    int rows;               // rows per wave of that variant (set by the launcher)
};

// Values that change from iteration to iteration, passed by value so that the
// argument blocks themselves can be read in place (kernarg or device table).
template <typename T>
struct Live {
    const T *zc, *zp;       // z(i-1), z(i-2)
    T *zn;                  // z(i) (in place of z(i-2))
    T beta, beta_next;      // momentum of y(i) and of y(i+1)
    double *slots;          // this iteration's statistic slots (nullptr: off)
};

// Per-iteration values of a lock-step batched launch.
template <typename T>
struct Dyn {
    T beta, beta_next;      // momentum of y(i) and of y(i+1)
    int parity;             // 1: the table's zc/zp are swapped this iteration
    int ring;               // statistics ring entry of this iteration
    const int *it_dev;      // replayed graph: beta, beta_next from i = *it_dev + it_off
    int it_off;
};

template <typename T> hipError_t launch_synth(const SynthArgs<T> &a, int C, hipStream_t s);
// Analysis levels D (a) and D + 1 (e) in one launch, gradient step + prox or
// plain mode, one channel per tile set; level D's approximation band stays in
// LDS (a.apx_out is not written).  Same outputs as two launch_analysis calls.
template <typename T>
hipError_t launch_analysis2(const AnalysisArgs<T> &a, const AnalysisArgs<T> &e, hipStream_t s);
// two synthesis levels in one launch: d = the finer level, u = the next coarser
// (its output, d's approximation band, stays in LDS; u.out is not written)
template <typename T>
hipError_t launch_synth2(const SynthArgs<T> &d, const SynthArgs<T> &u, int C, hipStream_t s);
// Levels D + 2, D + 1 and D in one launch (v, u, d), the same bits as three single-level launches
template <typename T>
hipError_t launch_synth3(const SynthArgs<T> &d, const SynthArgs<T> &u, const SynthArgs<T> &v, int C, hipStream_t s);
template <typename T> hipError_t launch_analysis(const AnalysisArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_coarse(const CoarseArgs<T> &a, int groups, hipStream_t s);
template <typename T> hipError_t launch_jprox(const JProxArgs<T> &a, int nch, hipStream_t s);
template <typename T> size_t coarse_lds_bytes(int m1, int m2, int chans);
template <typename T> hipError_t launch_blur(const BlurArgs<T> &a, bool identity, hipStream_t s);
template <typename T> hipError_t launch_blur_single(const BlurArgs<T> &a, int transpose, hipStream_t s);
template <typename T> hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_synth_b(const SynthArgs<T> *tab, const int *start, int n, int tiles, Dyn<T> d, hipStream_t s);
// nch = 0: scalar prox (tiles and coarse groups per channel); 1..4: joint prox
// over that many channels (tiles and coarse groups per image).
template <typename T>
hipError_t launch_analysis_b(const AnalysisArgs<T> *tab, const int *start, int n, int tiles, int nch, Dyn<T> d,
                             hipStream_t s);
template <typename T>
hipError_t launch_coarse_b(const CoarseArgs<T> *tab, const int *start, int n, int groups, size_t lds, int nch,
                           Dyn<T> d, hipStream_t s);
template <typename T>
hipError_t launch_blur_b(const BlurArgs<T> *tab, const int *start, int n, int tiles, int ring, hipStream_t s);
// The two marching kernels over many images (row blur, tables in a.tabs, r in
// a.r, a.rows = rows for every image): start_h / start_ht are the prefix sums
// of each image's workgroups (channels x a.tx for the r kernel, channels x a.ty
// for the H^T kernel, as tiles_blur_split gives them), wg_h / wg_ht their totals.
template <typename T>
hipError_t launch_blur_split_b(const BlurArgs<T> *tab, const int *start_h, const int *start_ht, int n, int wg_h,
                               int wg_ht, int rows, int ring, hipStream_t s);
void tiles_blur_split(int n1, int n2, int rows, int *th, int *tht);
// stats[it0+j][q] += sum of ring entry (it0+j) % PD_RING, then zeroed, for
// j < count; batched: one image per grid row, ring/stats bases from tables.
hipError_t launch_stats_finalize_b(double *const *ring, double *const *stats, int n, int it0, int count,
                                   const int *it_dev, hipStream_t s);  // it_dev: it0 += *it_dev
void tiles_synth(int M1c, int M2c, int *tx, int *ty);
void tiles_analysis(int M1c, int M2c, int *tx, int *ty);
void tiles_blur(int n1, int n2, int *tx, int *ty, int bt2 = 32);
// Blur variants (the tuned choice per size; 32 where nothing was tuned):
// 32, 48 = the fused tile kernel with that many output rows per workgroup;
// BLUR_SPLIT + w = the two marching kernels with w rows per wave (needs
// BlurArgs::r and ::tabs, else the fused 32-row kernel runs).  All variants
// give the same results bit for bit.
constexpr int BLUR_SPLIT = 1000;
// (rows + 2 PD_MAX_RADIUS a multiple of 2 PD_MAX_RADIUS + 1: no padded steps)
constexpr int BLUR_VARIANTS[] = {32, 48, BLUR_SPLIT + 20, BLUR_SPLIT + 39, BLUR_SPLIT + 58};
int blur_variant(int n1, int n2, int C, int R, int es);
void set_blur_variant(int n1, int n2, int C, int R, int es, int v);
// per-row profile tables of the two-kernel variant: tab = [2][n2][2 PD_MAX_RADIUS + 2]
template <typename T> hipError_t launch_blur_tables(const T *taps, int n2, int R, T *tab, hipStream_t s);
constexpr int BLUR_TAB_PITCH = 2 * PD_MAX_RADIUS + 2;
hipError_t launch_stats_finalize(double *ring, double *stats, int it0, int count, hipStream_t s);
// same with it0 = *it_dev - sub (graph replay)
hipError_t launch_stats_finalize_dev(double *ring, double *stats, const int *it_dev, int sub, int count, hipStream_t s);
hipError_t launch_set_int(int *dst, int v, hipStream_t s);
template <typename T> hipError_t launch_fill(T *dst, T v, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_rev_mask(const T *zbar, const T *z, T *vbar, T *wbar, T tau, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_rev_combine(const T *vbar, const T *gbar, T *zbar, T *zbarm, T tau, T b, int first, int64_t n,
                              DevIter di, hipStream_t s);
// launch_rev_combine of iteration i, then launch_rev_mask of iteration i-1 with z = z(i-1), in one launch;
// the sk2 x sk1 block at the top left of each plane (rows of `pitch`) is skipped (sk1 = 0: none)
template <typename T>
hipError_t launch_rev_combine_mask(T *vbar, const T *gbar, T *zbar, T *zbarm, const T *z, T *wbar, T tau, T b,
                                   int first, int64_t n, DevIter di, int sk1, int sk2, int pitch, int64_t plane,
                                   hipStream_t s);
template <typename T> hipError_t launch_add(const T *x, T *y, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_expand_weights(T *w, const T *wlev_dev, int n1, int n2, int C, int levels, hipStream_t s);

}  // namespace pd
