// pd_api.cpp -- the C ABI of libpd (include/pd.h): argument checks,
// workspace layout and the per-iteration launch sequence of FISTA-Spa
// (Escande & Weiss, arXiv:2005.09870, Appendix A.1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "pd.h"
#include "pd_kernels.h"

using namespace pd;

namespace {

inline size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

bool is_pow2_divisible(int n, int L) { return L >= 0 && L < 31 && (n % (1 << L)) == 0; }

int check_shape(const pd_shape *s)
{
    if (!s) return PD_ERR_ARG;
    if (s->n1 < 2 || s->n2 < 2 || s->channels < 1 || s->channels > PD_MAXC) return PD_ERR_SHAPE;
    if (s->levels < 1 || s->levels > PD_MAXL) return PD_ERR_SHAPE;
    if (!is_pow2_divisible(s->n1, s->levels) || !is_pow2_divisible(s->n2, s->levels)) return PD_ERR_SHAPE;
    if ((int64_t)s->n1 * s->n2 * s->channels > (int64_t)1 << 31) return PD_ERR_UNSUPPORTED;
    return PD_OK;
}

int check_dtype(int32_t dt) { return (dt == PD_F32 || dt == PD_F64) ? PD_OK : PD_ERR_ARG; }

int check_wavelet(const pd_wavelet *w)
{
    if (!w || !w->h) return PD_ERR_ARG;
    if (w->len < 2 || w->len > 12 || (w->len & 1)) return PD_ERR_UNSUPPORTED;
    for (int k = 0; k < w->len; ++k)
        if (!std::isfinite(w->h[k])) return PD_ERR_ARG;
    return PD_OK;
}

int check_op(const pd_operator *op, const pd_shape *s)
{
    if (!op) return PD_ERR_ARG;
    if (op->kind == PD_OP_IDENTITY) return PD_OK;
    if (op->kind != PD_OP_ROWBLUR) return PD_ERR_ARG;
    if (!op->taps) return PD_ERR_ARG;
    if (op->radius < 0 || op->radius > PD_MAX_RADIUS) return PD_ERR_UNSUPPORTED;
    (void)s;
    return PD_OK;
}

int check_weights(const pd_weights *w, const pd_shape *s)
{
    if (!w) return PD_ERR_ARG;
    if ((w->level_w == nullptr) == (w->coeff_w == nullptr)) return PD_ERR_ARG;
    if (w->joint && (w->coeff_w || s->channels < 1)) return PD_ERR_UNSUPPORTED;
    if (w->level_w)
        for (int k = 0; k <= s->levels; ++k)
            if (!std::isfinite(w->level_w[k]) || w->level_w[k] < 0.0) return PD_ERR_ARG;
    return PD_OK;
}

int check_params(const pd_params *p)
{
    if (!p) return PD_ERR_ARG;
    if (!std::isfinite(p->tau) || p->tau <= 0.0) return PD_ERR_TAU;
    if (p->iters < 0 || p->iter_offset < 0) return PD_ERR_ARG;
    return PD_OK;
}

template <typename T>
Filt<T> make_filt(const pd_wavelet *w)
{
    Filt<T> f;
    for (int k = 0; k < 12; ++k) f.h[k] = k < w->len ? (T)w->h[k] : T(0);
    for (int k = -10; k <= 1; ++k) {
        int m = 1 - k;  // g[k] = (-1)^(1-k) h[1-k]
        f.g[k + 10] = (m < w->len) ? (T)((m % 2 == 0 ? 1.0 : -1.0) * w->h[m]) : T(0);
    }
    return f;
}

// Workspace: approximation pyramid (levels 1..L-1), x, s, flag.
struct Layout {
    size_t apx[PD_MAXL + 1];
    size_t x, s, flag, total;
};

Layout layout(const pd_shape *s, size_t es)
{
    Layout l;
    size_t off = 0;
    const size_t C = s->channels;
    for (int j = 0; j <= PD_MAXL; ++j) l.apx[j] = 0;
    for (int j = 1; j < s->levels; ++j) {
        l.apx[j] = off;
        off = align_up(off + C * (size_t)(s->n1 >> j) * (size_t)(s->n2 >> j) * es);
    }
    const size_t plane = C * (size_t)s->n1 * s->n2 * es;
    l.x = off;
    off = align_up(off + plane);
    l.s = off;
    off = align_up(off + plane);
    l.flag = off;
    off = align_up(off + 256);
    l.total = off;
    return l;
}

#define PD_TRY_HIP(expr)                      \
    do {                                      \
        if ((expr) != hipSuccess) return PD_ERR_HIP; \
    } while (0)

template <typename T>
struct Ctx {
    const pd_shape *sh;
    Filt<T> f;
    char *ws;
    Layout lay;
    hipStream_t st;
    int64_t N() const { return (int64_t)sh->n1 * sh->n2; }
    T *apx(int j) const { return (T *)(ws + lay.apx[j]); }
    T *x() const { return (T *)(ws + lay.x); }
    T *s() const { return (T *)(ws + lay.s); }
    int *flag() const { return (int *)(ws + lay.flag); }
};

// x = Psi y, y = zc + beta (zc - zp)
template <typename T>
int synth_chain(const Ctx<T> &c, const T *zc, const T *zp, T beta, T *out)
{
    const int L = c.sh->levels, n1 = c.sh->n1, n2 = c.sh->n2;
    for (int lev = L; lev >= 1; --lev) {
        SynthArgs<T> a;
        a.f = c.f;
        a.zc = zc;
        a.zp = zp;
        a.beta = beta;
        a.plane = c.N();
        a.pitch = n1;
        a.apx = lev == L ? nullptr : c.apx(lev);
        a.apx_plane = (int64_t)(n1 >> lev) * (n2 >> lev);
        a.out = lev == 1 ? out : c.apx(lev - 1);
        a.out_pitch = lev == 1 ? n1 : (n1 >> (lev - 1));
        a.out_plane = lev == 1 ? c.N() : (int64_t)(n1 >> (lev - 1)) * (n2 >> (lev - 1));
        a.M1c = n1 >> lev;
        a.M2c = n2 >> lev;
        PD_TRY_HIP(launch_synth<T>(a, c.sh->channels, c.st));
    }
    return PD_OK;
}

// Forward transform of `in`: plain coefficients (mode PLAIN) or the fused
// gradient step + prox + momentum (mode PROX).
template <typename T>
int analysis_chain(const Ctx<T> &c, const T *in, int mode, const T *zc, const T *zp, T *zn,
                   T beta, T tau, const pd_weights *w, double *stats)
{
    const int L = c.sh->levels, n1 = c.sh->n1, n2 = c.sh->n2;
    for (int lev = 1; lev <= L; ++lev) {
        AnalysisArgs<T> a;
        a.f = c.f;
        a.in = lev == 1 ? in : c.apx(lev - 1);
        a.in_pitch = lev == 1 ? n1 : (n1 >> (lev - 1));
        a.in_plane = lev == 1 ? c.N() : (int64_t)(n1 >> (lev - 1)) * (n2 >> (lev - 1));
        a.M1c = n1 >> lev;
        a.M2c = n2 >> lev;
        a.last = lev == L;
        a.apx_out = lev < L ? c.apx(lev) : nullptr;
        a.apx_plane = (int64_t)(n1 >> lev) * (n2 >> lev);
        a.mode = mode;
        a.zc = zc;
        a.zp = zp;
        a.zn = zn;
        a.beta = beta;
        a.tau = tau;
        a.plane = c.N();
        a.pitch = n1;
        a.wmap = nullptr;
        for (int k = 0; k <= PD_MAXL; ++k) a.wlev[k] = T(0);
        a.joint = 0;
        if (w) {
            a.wmap = (const T *)w->coeff_w;
            if (w->level_w)
                for (int k = 0; k <= L; ++k) a.wlev[k] = (T)w->level_w[k];
            a.joint = w->joint ? 1 : 0;
        }
        a.band_detail = L + 1 - lev;
        a.C = c.sh->channels;
        a.stats = stats;
        a.flag = c.flag();
        PD_TRY_HIP(launch_analysis<T>(a, c.st));
    }
    return PD_OK;
}

template <typename T>
int blur_step(const Ctx<T> &c, const pd_operator *op, const T *x, const T *f0, T *s, double *stats)
{
    BlurArgs<T> a;
    a.x = x;
    a.f0 = f0;
    a.s = s;
    a.taps = (const T *)op->taps;
    a.n1 = c.sh->n1;
    a.n2 = c.sh->n2;
    a.C = c.sh->channels;
    a.R = op->radius;
    a.plane = c.N();
    a.stats = stats;
    PD_TRY_HIP(launch_blur<T>(a, op->kind == PD_OP_IDENTITY, c.st));
    return PD_OK;
}

template <typename T>
int solve_impl(const pd_shape *sh, const pd_operator *op, const pd_wavelet *wav, const pd_weights *w,
               const pd_params *prm, const T *f0, T *z_cur, T *z_prev, int init, T *f_out,
               double *stats, void *workspace, size_t ws_bytes, hipStream_t st)
{
    Ctx<T> c;
    c.sh = sh;
    c.f = make_filt<T>(wav);
    c.ws = (char *)workspace;
    c.lay = layout(sh, sizeof(T));
    c.st = st;
    if (ws_bytes < c.lay.total) return PD_ERR_WORKSPACE;
    const int64_t NC = c.N() * sh->channels;
    int rc;
    if (init) {
        if ((rc = analysis_chain<T>(c, f0, MODE_PLAIN, nullptr, nullptr, z_cur, T(0), T(0), nullptr,
                                    nullptr)) != PD_OK)
            return rc;
        PD_TRY_HIP(launch_copy<T>(z_cur, z_prev, NC, st));
    }
    if (prm->check_finite) PD_TRY_HIP(hipMemsetAsync(c.flag(), 0, sizeof(int), st));
    T *zc = z_cur, *zp = z_prev;
    const T tau = (T)prm->tau;
    for (int it = 0; it < prm->iters; ++it) {
        const int i = prm->iter_offset + 1 + it;  // global iteration number
        // y(i) = z(i-1) + b_{i-1} (z(i-1) - z(i-2)),  b_k = (k-1)/(k+2)
        const T beta = i >= 2 ? (T)((double)(i - 2) / (double)(i + 1)) : T(0);
        double *sti = stats ? stats + 3 * (size_t)it : nullptr;
        if ((rc = synth_chain<T>(c, zc, zp, beta, c.x())) != PD_OK) return rc;
        if ((rc = blur_step<T>(c, op, c.x(), f0, c.s(), sti)) != PD_OK) return rc;
        // z(i) overwrites z(i-2) in place (each coefficient read then written by one thread)
        if ((rc = analysis_chain<T>(c, c.s(), MODE_PROX, zc, zp, zp, beta, tau, w, sti)) != PD_OK)
            return rc;
        T *t = zc;
        zc = zp;
        zp = t;
    }
    if (zc != z_cur) {  // odd number of iterations: swap the two planes
        T *tmp = c.x();
        PD_TRY_HIP(launch_copy<T>(z_cur, tmp, NC, st));
        PD_TRY_HIP(launch_copy<T>(z_prev, z_cur, NC, st));
        PD_TRY_HIP(launch_copy<T>(tmp, z_prev, NC, st));
    }
    if (f_out)
        if ((rc = synth_chain<T>(c, z_cur, z_cur, T(0), f_out)) != PD_OK) return rc;
    if (prm->check_finite) {
        int h = 0;
        PD_TRY_HIP(hipMemcpyAsync(&h, c.flag(), sizeof(int), hipMemcpyDeviceToHost, st));
        PD_TRY_HIP(hipStreamSynchronize(st));
        if (h) return PD_ERR_NONFINITE;
    }
    return PD_OK;
}

}  // namespace

extern "C" size_t pd_workspace_size(const pd_shape *shape, int32_t dtype)
{
    if (check_shape(shape) != PD_OK || check_dtype(dtype) != PD_OK) return 0;
    return layout(shape, dtype == PD_F64 ? 8 : 4).total;
}

extern "C" int pd_solve(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                        const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                        const void *f0, void *z_cur, void *z_prev, int32_t init_from_f0,
                        void *f_out, double *stats, void *workspace, size_t ws_bytes,
                        void *stream)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype)) || (rc = check_op(op, shape)) ||
        (rc = check_wavelet(wav)) || (rc = check_weights(w, shape)) || (rc = check_params(prm)))
        return rc;
    if (!f0 || !z_cur || !z_prev || !workspace || z_cur == z_prev) return PD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PD_F32)
        return solve_impl<float>(shape, op, wav, w, prm, (const float *)f0, (float *)z_cur,
                                 (float *)z_prev, init_from_f0, (float *)f_out, stats, workspace,
                                 ws_bytes, st);
    return solve_impl<double>(shape, op, wav, w, prm, (const double *)f0, (double *)z_cur,
                              (double *)z_prev, init_from_f0, (double *)f_out, stats, workspace,
                              ws_bytes, st);
}

extern "C" int pd_fwt(const pd_shape *shape, int32_t dtype, const pd_wavelet *wav, int32_t inverse,
                      const void *in, void *out, void *workspace, size_t ws_bytes, void *stream)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype)) || (rc = check_wavelet(wav)))
        return rc;
    if (!in || !out || !workspace || in == out) return PD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        Ctx<T> c;
        c.sh = shape;
        c.f = make_filt<T>(wav);
        c.ws = (char *)workspace;
        c.lay = layout(shape, sizeof(T));
        c.st = st;
        if (ws_bytes < c.lay.total) return PD_ERR_WORKSPACE;
        if (inverse) return synth_chain<T>(c, (const T *)in, (const T *)in, T(0), (T *)out);
        return analysis_chain<T>(c, (const T *)in, MODE_PLAIN, nullptr, nullptr, (T *)out, T(0),
                                 T(0), nullptr, nullptr);
    };
    return dtype == PD_F32 ? run(float(0)) : run(double(0));
}

extern "C" int pd_apply_op(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                           int32_t transpose, const void *in, void *out, void *stream)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype)) || (rc = check_op(op, shape)))
        return rc;
    if (!in || !out || in == out) return PD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int64_t NC = (int64_t)shape->n1 * shape->n2 * shape->channels;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        if (op->kind == PD_OP_IDENTITY) {
            PD_TRY_HIP(launch_copy<T>((const T *)in, (T *)out, NC, st));
            return PD_OK;
        }
        BlurArgs<T> a;
        a.x = (const T *)in;
        a.f0 = nullptr;
        a.s = (T *)out;
        a.taps = (const T *)op->taps;
        a.n1 = shape->n1;
        a.n2 = shape->n2;
        a.C = shape->channels;
        a.R = op->radius;
        a.plane = (int64_t)shape->n1 * shape->n2;
        a.stats = nullptr;
        PD_TRY_HIP(launch_blur_single<T>(a, transpose, st));
        return PD_OK;
    };
    return dtype == PD_F32 ? run(float(0)) : run(double(0));
}

// ---------------------------------------------------------------- batched --
extern "C" size_t pd_batched_workspace_size(int32_t batch, const pd_image_desc *descs, int32_t dtype)
{
    if (batch < 1 || !descs || check_dtype(dtype) != PD_OK) return 0;
    size_t mx = 0;
    for (int b = 0; b < batch; ++b) {
        if (check_shape(&descs[b].shape) != PD_OK) return 0;
        size_t es = dtype == PD_F64 ? 8 : 4;
        size_t need = layout(&descs[b].shape, es).total +
                      align_up(es * descs[b].shape.channels * (size_t)descs[b].shape.n1 * descs[b].shape.n2);
        mx = need > mx ? need : mx;
    }
    return mx;
}

extern "C" int pd_solve_batched(int32_t batch, const pd_image_desc *descs, int32_t dtype,
                                const pd_wavelet *wav, int32_t iters, const void *f0_packed,
                                void *f_out_packed, double *stats, void *workspace,
                                size_t ws_bytes, void *stream)
{
    int rc;
    if (batch < 1 || !descs || !f0_packed || !f_out_packed || !workspace || iters < 0) return PD_ERR_ARG;
    if ((rc = check_dtype(dtype)) || (rc = check_wavelet(wav))) return rc;
    for (int b = 0; b < batch; ++b) {
        const pd_image_desc &d = descs[b];
        if ((rc = check_shape(&d.shape)) || (rc = check_op(&d.op, &d.shape))) return rc;
        if (!d.level_w || d.offset < 0) return PD_ERR_ARG;
        if (!std::isfinite(d.tau) || d.tau <= 0.0) return PD_ERR_TAU;
    }
    if (ws_bytes < pd_batched_workspace_size(batch, descs, dtype)) return PD_ERR_WORKSPACE;
    // per-image loop over the single-image path: z(i-1) lives in f_out, z(i-2) in the workspace tail
    const size_t es = dtype == PD_F64 ? 8 : 4;
    for (int b = 0; b < batch; ++b) {
        const pd_image_desc &d = descs[b];
        const size_t lay = layout(&d.shape, es).total;
        char *zprev = (char *)workspace + lay;
        char *zc = (char *)f_out_packed + d.offset * es;
        const char *f0 = (const char *)f0_packed + d.offset * es;
        pd_weights w{d.level_w, nullptr, 0};
        pd_params p{d.tau, iters, 0, 0};
        double *sb = stats ? stats + (size_t)b * iters * 3 : nullptr;
        rc = pd_solve(&d.shape, dtype, &d.op, wav, &w, &p, f0, zc, zprev, 1, nullptr, sb,
                      workspace, lay, stream);
        if (rc) return rc;
        // f = Psi z in place via the x buffer
        Layout l = layout(&d.shape, es);
        char *x = (char *)workspace + l.x;
        rc = pd_fwt(&d.shape, dtype, wav, 1, zc, x, workspace, lay, stream);
        if (rc) return rc;
        const int64_t NC = (int64_t)d.shape.n1 * d.shape.n2 * d.shape.channels;
        if (dtype == PD_F32)
            PD_TRY_HIP(launch_copy<float>((const float *)x, (float *)zc, NC, (hipStream_t)stream));
        else
            PD_TRY_HIP(launch_copy<double>((const double *)x, (double *)zc, NC, (hipStream_t)stream));
    }
    return PD_OK;
}

// --------------------------------------------------------------- backward --
extern "C" size_t pd_backward_workspace_size(const pd_shape *shape, int32_t dtype, int32_t iters,
                                             int32_t checkpoint_every)
{
    (void)shape;
    (void)dtype;
    (void)iters;
    (void)checkpoint_every;
    return 0;
}

extern "C" int pd_backward(const pd_shape *, int32_t, const pd_operator *, const pd_wavelet *,
                           const pd_weights *, const pd_params *, const void *, const void *,
                           void *, void *, int32_t, void *, size_t, void *)
{
    return PD_ERR_UNSUPPORTED;
}
