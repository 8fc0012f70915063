// pd_kernels.h -- argument blocks and launchers of the gfx950 kernels
// (internal to libpd; the public interface is include/pd.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#define PD_MAXC 4
#define PD_MAXL 16
#define PD_MAX_RADIUS 9

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
template <typename T>
struct SynthArgs {
    Filt<T> f;
    const T *zc, *zp;
    T beta;
    int64_t plane;
    int pitch;
    const T *apx;
    int64_t apx_plane;
    T *out;
    int out_pitch;
    int64_t out_plane;
    int M1c, M2c;
};

enum { MODE_PLAIN = 0, MODE_PROX = 1 };

// One analysis level: fine input M1 x M2 -> four coarse M1c x M2c bands.
// MODE_PLAIN stores the detail bands (and, if last, the approximation band)
// of the input in zn.  MODE_PROX treats them as the gradient g and stores
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
    const T *zc, *zp;
    T *zn;
    T beta, tau;
    int64_t plane;
    int pitch;
    const T *wmap;          // per-coefficient weights or nullptr
    T wlev[PD_MAXL + 1];    // per-band weights
    int band_detail;        // band index k of this level's detail bands
    int joint, C;
    double *stats;          // [sum w|y|, sum (z-y)^2] at stats+1, stats+2
    int *flag;              // set to 1 if a prox argument is not finite
};

// Fused r = H x - f0, s = H^T r (or a single pass for the building block).
template <typename T>
struct BlurArgs {
    const T *x, *f0;
    T *s;
    const T *taps;
    int n1, n2, C, R;
    int64_t plane;
    double *stats;          // 1/2 ||r||^2 at stats[0]
};

template <typename T> hipError_t launch_synth(const SynthArgs<T> &a, int C, hipStream_t s);
template <typename T> hipError_t launch_analysis(const AnalysisArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_blur(const BlurArgs<T> &a, bool identity, hipStream_t s);
template <typename T> hipError_t launch_blur_single(const BlurArgs<T> &a, int transpose, hipStream_t s);
template <typename T> hipError_t launch_copy(const T *src, T *dst, int64_t n, hipStream_t s);

}  // namespace pd
