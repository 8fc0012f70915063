// pd_pckernels.h -- argument block and launchers of the gfx950 kernels of the
// product-convolution operator H f = sum_k u_k * (v_k . f) (Section 1's
// expansion, Section 3.1; FISTA-PC of Table 1).  Internal to libpd.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pd_kernels.h"

#define PD_MAX_PC 64  // terms of an expansion

namespace pd {

// u: [m][2R+1][2R+1] kernels (row-major in (d2, d1), d in [-R, R]^2);
// v: [m][n2][n1] multipliers, shared by the channels.
// Fused (f0 != nullptr or slots): r = H x - f0 (1/2||r||^2 to slots row 0),
// s = H^T r; single pass: s = H x or H^T x.
template <typename T>
struct PcArgs {
    const T *x, *f0;
    T *s;
    const T *u, *v;
    int n1, n2, C, R, m;
    int64_t plane;
    double *slots;
};

template <typename T> hipError_t launch_pcblur(const PcArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_pc_single(const PcArgs<T> &a, int transpose, hipStream_t s);

}  // namespace pd
