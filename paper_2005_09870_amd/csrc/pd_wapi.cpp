// pd_wapi.cpp -- the C ABI of FISTA in the wavelet domain (FISTA-W and
// FISTA-WP, Section 4.3 and Appendix A.1 of Escande & Weiss,
// arXiv:2005.09870): argument checks, workspace layout, the two-launch
// iteration, and the CSR set-up calls (transpose, product, Jacobi diagonal).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <utility>

#include "pd.h"
#include "pd_internal.h"
#include "pd_kernels.h"
#include "pd_wkernels.h"

using namespace pd;

namespace {

int check_csr(const pd_csr *a)
{
    if (!a || !a->row_ptr || a->n < 1 || a->nnz < 0) return PD_ERR_ARG;
    if (a->nnz > 0 && (!a->col || !a->val)) return PD_ERR_ARG;
    return PD_OK;
}

template <typename T>
Csr<T> view(const pd_csr *a)
{
    return Csr<T>{a->row_ptr, a->col, (const T *)a->val, a->n, a->nnz};
}

// Workspace of pd_wsolve: u, sigma, y (n each), flag, statistics ring.
struct WLayout {
    size_t u, sigma, y, flag, ring, total;
};

WLayout wlayout(int64_t n, size_t es)
{
    WLayout l;
    size_t off = 0;
    l.u = off;
    off = align_up(off + n * es);
    l.sigma = off;
    off = align_up(off + n * es);
    l.y = off;
    off = align_up(off + n * es);
    l.flag = off;
    off = align_up(off + 256);
    l.ring = off;
    off = align_up(off + (size_t)PD_RING * 3 * PD_NSLOT * sizeof(double));
    l.total = off;
    return l;
}

int check_wshape(const pd_shape *s)
{
    if (!s) return PD_ERR_ARG;
    if (s->n1 < 2 || s->n2 < 2 || s->channels != 1) return PD_ERR_SHAPE;
    if (s->levels < 1 || s->levels > PD_MAXL) return PD_ERR_SHAPE;
    if (s->n1 % (1 << s->levels) || s->n2 % (1 << s->levels)) return PD_ERR_SHAPE;
    if ((int64_t)s->n1 * s->n2 > ((int64_t)1 << 31) - 1) return PD_ERR_UNSUPPORTED;
    return PD_OK;
}

// Momentum of y(i) = z(i-1) + b (z(i-1) - z(i-2)):  b = (i-2)/(i+1), 0 for i = 1.
inline double wbeta_y(int i) { return i >= 2 ? (double)(i - 2) / (double)(i + 1) : 0.0; }

template <typename T>
int wsolve_impl(const pd_shape *sh, const pd_csr *th, const pd_csr *tht, const pd_weights *w,
                const pd_params *prm, int precond, const T *z0, T *z_cur, T *z_prev, int init, double *stats,
                void *workspace, size_t ws_bytes, hipStream_t st)
{
    const int64_t n = th->n;
    const WLayout L = wlayout(n, sizeof(T));
    if (ws_bytes < L.total) return PD_ERR_WORKSPACE;
    char *ws = (char *)workspace;
    T *u = (T *)(ws + L.u), *sigma = (T *)(ws + L.sigma), *y = (T *)(ws + L.y);
    int *flag = (int *)(ws + L.flag);
    double *ring = (double *)(ws + L.ring);
    const Csr<T> A = view<T>(th), At = view<T>(tht);
    const int gA = wgroup_for(th->nnz, th->n), gT = wgroup_for(tht->nnz, tht->n);

    if (init) {
        PD_TRY_HIP(launch_copy<T>(z0, z_cur, n, st));
        PD_TRY_HIP(launch_copy<T>(z0, z_prev, n, st));
    }
    if (prm->check_finite) PD_TRY_HIP(launch_fill_i32(flag, 0, 1, st));
    if (precond) PD_TRY_HIP(launch_wjacobi<T>(At, sigma, gT, st));
    const int K = prm->iters, i0 = prm->iter_offset + 1;
    if (K > 0) PD_TRY_HIP(launch_wform_y<T>(z_cur, z_prev, (T)wbeta_y(i0), y, n, st));
    if (stats && K > 0) PD_TRY_HIP(launch_fill<double>(ring, 0.0, (int64_t)PD_RING * 3 * PD_NSLOT, st));

    WResArgs<T> ra{A, y, z0, u, nullptr};
    WProxArgs<T> pa{};
    pa.at = At;
    pa.u = u;
    pa.y = y;
    pa.sigma = precond ? sigma : nullptr;
    pa.wmap = (const T *)w->coeff_w;
    for (int k = 0; k <= PD_MAXL; ++k) pa.wlev[k] = (w->level_w && k <= sh->levels) ? (T)w->level_w[k] : T(0);
    pa.n1 = sh->n1;
    pa.n2 = sh->n2;
    pa.levels = sh->levels;
    pa.tau = (T)prm->tau;
    pa.flag = flag;

    T *zc = z_cur, *zp = z_prev;
    for (int it = 0; it < K; ++it) {
        const int i = i0 + it;
        double *sl = stats ? ring + (size_t)(it % PD_RING) * 3 * PD_NSLOT : nullptr;
        ra.slots = sl;
        PD_TRY_HIP(timed(PD_K_WRES, 0, st, [&] { return launch_wres<T>(ra, gA, st); }));
        pa.zc = zc;
        pa.zn = zp;  // z(i) in place of z(i-2)
        pa.beta_next = (T)wbeta_y(i + 1);
        pa.slots = sl;
        PD_TRY_HIP(timed(PD_K_WPROX, 0, st, [&] { return launch_wprox<T>(pa, gT, st); }));
        std::swap(zc, zp);
        if (stats && ((it + 1) % PD_RING == 0 || it == K - 1)) {
            const int cnt = (it % PD_RING) + 1;
            PD_TRY_HIP(launch_stats_finalize(ring, stats, it + 1 - cnt, cnt, st));
        }
    }
    if (zc != z_cur) {  // odd number of iterations: swap the two planes (u is free now)
        PD_TRY_HIP(launch_copy<T>(z_cur, u, n, st));
        PD_TRY_HIP(launch_copy<T>(z_prev, z_cur, n, st));
        PD_TRY_HIP(launch_copy<T>(u, z_prev, n, st));
    }
    if (prm->check_finite) {
        int h = 0;
        PD_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
        PD_TRY_HIP(hipStreamSynchronize(st));
        if (h) return PD_ERR_NONFINITE;
    }
    return PD_OK;
}

template <typename T>
int transpose_impl(const pd_csr *a, int64_t *trp, int32_t *tcol, T *tval, void *workspace, hipStream_t st)
{
    const int n = a->n;
    int *cnt = (int *)workspace;
    int *cur = cnt + n;
    int *flag = (int *)((char *)workspace + align_up(2 * (size_t)n * sizeof(int)));
    PD_TRY_HIP(launch_fill_i32(flag, 0, 1, st));
    PD_TRY_HIP(launch_csr_check(a->row_ptr, a->col, n, a->nnz, flag, st));
    int h = 0;
    PD_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    PD_TRY_HIP(hipStreamSynchronize(st));
    if (h) return PD_ERR_ARG;
    PD_TRY_HIP(launch_fill_i32(cnt, 0, 2 * (int64_t)n, st));
    PD_TRY_HIP(launch_csr_count(a->row_ptr, a->col, n, cnt, st));
    PD_TRY_HIP(launch_csr_scan(cnt, n, trp, st));
    PD_TRY_HIP(launch_csr_scatter<T>(view<T>(a), trp, cur, tcol, tval, st));
    PD_TRY_HIP(launch_csr_sort<T>(trp, n, tcol, tval, st));
    return PD_OK;
}

}  // namespace

extern "C" size_t pd_csr_transpose_workspace_size(int32_t n)
{
    if (n < 1) return 0;
    return align_up(2 * (size_t)n * sizeof(int)) + 256;
}

extern "C" int pd_csr_transpose(const pd_csr *a, int32_t dtype, int64_t *t_row_ptr, int32_t *t_col, void *t_val,
                                void *workspace, size_t ws_bytes, void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    int rc;
    if ((rc = check_csr(a)) != PD_OK) return rc;
    if (dtype != PD_F32 && dtype != PD_F64) return PD_ERR_ARG;
    if (!t_row_ptr || (a->nnz > 0 && (!t_col || !t_val)) || !workspace) return PD_ERR_ARG;
    if (ws_bytes < pd_csr_transpose_workspace_size(a->n)) return PD_ERR_WORKSPACE;
    return dtype == PD_F32 ? transpose_impl<float>(a, t_row_ptr, t_col, (float *)t_val, workspace, stream)
                           : transpose_impl<double>(a, t_row_ptr, t_col, (double *)t_val, workspace, stream);
}

extern "C" int pd_spmv(const pd_csr *a, int32_t dtype, const void *x, void *y, void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    int rc;
    if ((rc = check_csr(a)) != PD_OK) return rc;
    if (!x || !y) return PD_ERR_ARG;
    const int g = wgroup_for(a->nnz, a->n);
    if (dtype == PD_F32) {
        WResArgs<float> r{view<float>(a), (const float *)x, nullptr, (float *)y, nullptr};
        PD_TRY_HIP(launch_wres<float>(r, g, stream));
    } else if (dtype == PD_F64) {
        WResArgs<double> r{view<double>(a), (const double *)x, nullptr, (double *)y, nullptr};
        PD_TRY_HIP(launch_wres<double>(r, g, stream));
    } else {
        return PD_ERR_ARG;
    }
    return PD_OK;
}

extern "C" int pd_wjacobi(const pd_csr *theta_t, int32_t dtype, void *sigma, void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    int rc;
    if ((rc = check_csr(theta_t)) != PD_OK) return rc;
    if (!sigma) return PD_ERR_ARG;
    const int g = wgroup_for(theta_t->nnz, theta_t->n);
    if (dtype == PD_F32)
        PD_TRY_HIP(launch_wjacobi<float>(view<float>(theta_t), (float *)sigma, g, stream));
    else if (dtype == PD_F64)
        PD_TRY_HIP(launch_wjacobi<double>(view<double>(theta_t), (double *)sigma, g, stream));
    else
        return PD_ERR_ARG;
    return PD_OK;
}

extern "C" size_t pd_wsolve_workspace_size(const pd_shape *shape, int32_t dtype)
{
    if (check_wshape(shape) != PD_OK || (dtype != PD_F32 && dtype != PD_F64)) return 0;
    return wlayout((int64_t)shape->n1 * shape->n2, dtype == PD_F32 ? 4 : 8).total;
}

extern "C" int pd_wsolve(const pd_shape *shape, int32_t dtype, const pd_csr *theta, const pd_csr *theta_t,
                         const pd_weights *w, const pd_params *prm, int32_t precond, const void *z0, void *z_cur,
                         void *z_prev, int32_t init_from_z0, double *stats, void *workspace, size_t ws_bytes,
                         void *stream_)
{
    const hipStream_t stream = (hipStream_t)stream_;
    int rc;
    if ((rc = check_wshape(shape)) != PD_OK) return rc;
    if (dtype != PD_F32 && dtype != PD_F64) return PD_ERR_ARG;
    if ((rc = check_csr(theta)) != PD_OK || (rc = check_csr(theta_t)) != PD_OK) return rc;
    const int64_t n = (int64_t)shape->n1 * shape->n2;
    if (theta->n != n || theta_t->n != n) return PD_ERR_SHAPE;
    if (!w || (w->level_w == nullptr) == (w->coeff_w == nullptr) || w->joint) return PD_ERR_ARG;
    if (w->level_w)
        for (int k = 0; k <= shape->levels; ++k)
            if (!std::isfinite(w->level_w[k]) || w->level_w[k] < 0.0) return PD_ERR_ARG;
    if (!prm) return PD_ERR_ARG;
    if (!std::isfinite(prm->tau) || prm->tau <= 0.0) return PD_ERR_TAU;
    if (prm->iters < 0 || prm->iter_offset < 0) return PD_ERR_ARG;
    if (!z0 || !z_cur || !z_prev || !workspace) return PD_ERR_ARG;
    if (z_cur == z_prev || z0 == z_cur || z0 == z_prev) return PD_ERR_ARG;  // aliased state
    if (dtype == PD_F32)
        return wsolve_impl<float>(shape, theta, theta_t, w, prm, precond != 0, (const float *)z0, (float *)z_cur,
                                  (float *)z_prev, init_from_z0, stats, workspace, ws_bytes, stream);
    return wsolve_impl<double>(shape, theta, theta_t, w, prm, precond != 0, (const double *)z0, (double *)z_cur,
                               (double *)z_prev, init_from_z0, stats, workspace, ws_bytes, stream);
}
