// pd_api.cpp -- the C ABI of libpd (include/pd.h): argument checks,
// workspace layout and the per-iteration launch sequence of FISTA-Spa
// (Escande & Weiss, arXiv:2005.09870, Appendix A.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>
#include <utility>
#include <vector>
#include <mutex>
#include <thread>

#include "pd.h"
#include "pd_internal.h"
#include "pd_kernels.h"
#include "pd_pckernels.h"
#include "pd_admm.h"
#include "pd_decomp.h"

using namespace pd;

namespace {

bool g_synth2 = true;  // the coarsest fine synthesis levels (three, or two) in one launch (pd_fuse_enable)

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
    if (op->kind != PD_OP_ROWBLUR && op->kind != PD_OP_PC) return PD_ERR_ARG;
    if (!op->taps) return PD_ERR_ARG;
    if (op->radius < 0 || op->radius > PD_MAX_RADIUS) return PD_ERR_UNSUPPORTED;
    if (op->kind == PD_OP_PC) {
        if (!op->mult || op->terms < 1) return PD_ERR_ARG;
        if (op->terms > PD_MAX_PC) return PD_ERR_UNSUPPORTED;
    }
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

// Workspace: approximation pyramid (levels 1..L-1), x, s, r (the two-kernel
// blur's intermediate), the blur's profile tables, flag, statistics ring,
// tail matrices, graph iteration number.
struct Layout {
    size_t apx[PD_MAXL + 1];
    size_t x, s, r, btab, flag, slots, tail, it, total;
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
    l.r = off;
    off = align_up(off + plane);
    l.btab = off;
    off = align_up(off + 2 * (size_t)s->n2 * BLUR_TAB_PITCH * es);
    l.flag = off;
    off = align_up(off + 256);
    l.slots = off;
    off = align_up(off + (size_t)PD_RING * 3 * PD_NSLOT * sizeof(double));
    l.tail = off;
    off = align_up(off + 2 * PD_TAIL_MAX * PD_TAIL_MAX * es);
    l.it = off;  // device iteration number of replayed graphs
    off = align_up(off + 256);
    l.total = off;
    return l;
}


// Largest approximation (per side) the coarse kernel holds in LDS.
constexpr int COARSE_MAX = 64;
constexpr size_t COARSE_LDS_MAX = 156 * 1024;

// The coarse block's last levels (input <= PD_TAIL_MAX values) are applied as
// one orthogonal matrix.  kw = levels done pass by pass before the tail.
struct TailShape {
    int kw, tM1, tM2, nt;
};

TailShape tail_shape(int m1, int m2, int nlev)
{
    TailShape t{0, m1, m2, nlev};
    while (t.kw < nlev && (m1 >> t.kw) * (m2 >> t.kw) > PD_TAIL_MAX) ++t.kw;
    t.tM1 = m1 >> t.kw;
    t.tM2 = m2 >> t.kw;
    t.nt = nlev - t.kw;
    return t;
}

template <typename T>
struct Ctx {
    const pd_shape *sh;
    Filt<T> f;
    char *ws;
    Layout lay;
    hipStream_t st;
    int lc;  // first level handled by the coarse kernel (levels + 1: none)
    bool eager = false;  // no graph replay (the allocation-free entry point)
    TailShape ts;
    const T *tail;  // device copy of the tail matrices (nullptr: none)
    const T *btab = nullptr;  // the blur's profile tables once filled (prep_blur)
    int64_t N() const { return (int64_t)sh->n1 * sh->n2; }
    T *apx(int j) const { return (T *)(ws + lay.apx[j]); }
    T *x() const { return (T *)(ws + lay.x); }
    T *s() const { return (T *)(ws + lay.s); }
    int *flag() const { return (int *)(ws + lay.flag); }
    double *ring() const { return (double *)(ws + lay.slots); }
    double *slots(int it) const { return ring() + (size_t)(it % PD_RING) * 3 * PD_NSLOT; }
    int *it_dev() const { return (int *)(ws + lay.it); }
};

// First level lc such that the level lc-1 approximation fits the coarse
// kernel (<= COARSE_MAX per side and its LDS budget); levels+1 if none.
template <typename T>
int coarse_level(const pd_shape *sh, int joint)
{
    const int chans = joint ? sh->channels : 1;
    for (int lc = 1; lc <= sh->levels; ++lc) {
        int m1 = sh->n1 >> (lc - 1), m2 = sh->n2 >> (lc - 1);
        if (m1 <= COARSE_MAX && m2 <= COARSE_MAX &&
            coarse_lds_bytes<T>(m1, m2, chans) <= COARSE_LDS_MAX)
            return lc;
    }
    return sh->levels + 1;
}

// Host analysis (Sections 2.1-2.2, same index conventions as the kernels) of
// a tM2 x tM1 array over nt levels, in place.
void host_analysis(std::vector<double> &x, int M1, int M2, int nt, const Filt<double> &f)
{
    int m1 = M1, m2 = M2;
    std::vector<double> t(std::max(M1, M2));
    auto md = [](int a, int n) { int r = a % n; return r < 0 ? r + n : r; };
    for (int lev = 0; lev < nt; ++lev) {
        for (int r = 0; r < m2; ++r) {
            for (int l = 0; l < m1 / 2; ++l) {
                double lo = 0.0, hi = 0.0;
                for (int k = 0; k < 12; ++k) {
                    lo += f.h[k] * x[(size_t)r * M1 + md(2 * l + k, m1)];
                    hi += f.g[k] * x[(size_t)r * M1 + md(2 * l + k - 10, m1)];
                }
                t[l] = lo;
                t[m1 / 2 + l] = hi;
            }
            for (int c = 0; c < m1; ++c) x[(size_t)r * M1 + c] = t[c];
        }
        for (int c = 0; c < m1; ++c) {
            for (int l = 0; l < m2 / 2; ++l) {
                double lo = 0.0, hi = 0.0;
                for (int k = 0; k < 12; ++k) {
                    lo += f.h[k] * x[(size_t)md(2 * l + k, m2) * M1 + c];
                    hi += f.g[k] * x[(size_t)md(2 * l + k - 10, m2) * M1 + c];
                }
                t[l] = lo;
                t[m2 / 2 + l] = hi;
            }
            for (int r = 0; r < m2; ++r) x[(size_t)r * M1 + c] = t[r];
        }
        m1 /= 2;
        m2 /= 2;
    }
}

// [2][tn][tn]: the tail's analysis matrix (row i = output i) and its transpose.
// Cached per (shape, filter, dtype); the cache keeps the host copy alive for
// asynchronous uploads.
std::mutex g_tail_mu;

template <typename T>
const std::vector<T> &tail_matrices(const TailShape &ts, const pd_wavelet *wav)
{
    static std::map<std::vector<double>, std::vector<T>> cache;  // entries are never erased
    std::lock_guard<std::mutex> lk(g_tail_mu);
    std::vector<double> key{(double)ts.tM1, (double)ts.tM2, (double)ts.nt};
    for (int k = 0; k < wav->len; ++k) key.push_back(wav->h[k]);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int tn = ts.tM1 * ts.tM2;
    const Filt<double> f = make_filt<double>(wav);
    std::vector<T> m(2 * (size_t)tn * tn);
    std::vector<double> x(tn);
    for (int j = 0; j < tn; ++j) {
        std::fill(x.begin(), x.end(), 0.0);
        x[j] = 1.0;
        host_analysis(x, ts.tM1, ts.tM2, ts.nt, f);
        for (int i = 0; i < tn; ++i) {
            m[(size_t)i * tn + j] = (T)x[i];                      // analysis: out i <- in j
            m[(size_t)tn * tn + (size_t)j * tn + i] = (T)x[i];    // transpose
        }
    }
    return cache.emplace(key, std::move(m)).first->second;
}

template <typename T>
ProxArgs<T> prox_args(const Ctx<T> &c, const T *zc, const T *zp, T *zn, T beta, T tau,
                      const pd_weights *w, double *slots)
{
    ProxArgs<T> p;
    p.zc = zc;
    p.zp = zp;
    p.zn = zn;
    p.zsave = nullptr;
    p.beta = beta;
    p.tau = tau;
    p.plane = c.N();
    p.pitch = c.sh->n1;
    p.wmap = nullptr;
    for (int k = 0; k <= PD_MAXL; ++k) p.wlev[k] = T(0);
    p.joint = 0;
    if (w) {
        p.wmap = (const T *)w->coeff_w;
        if (w->level_w)
            for (int k = 0; k <= c.sh->levels; ++k) p.wlev[k] = (T)w->level_w[k];
        p.joint = w->joint ? 1 : 0;
    }
    p.C = c.sh->channels;
    p.slots = slots;
    p.flag = c.flag();
    p.di = DevIter{nullptr, 0};
    return p;
}

// Coarse kernel: ops = COARSE_* bits.  Analysis input is the level lc-1
// approximation (apx[lc-1], or `in` when lc == 1); synthesis output goes to
// apx[lc-1] or `out` when lc == 1.
template <typename T>
int coarse_step(const Ctx<T> &c, int ops, const T *in, T *out, const ProxArgs<T> &p, T beta_next,
                const CoarseArgs<T> *rv = nullptr)
{
    const int L = c.sh->levels, lc = c.lc;
    CoarseArgs<T> a;
    a.f = c.f;
    a.ops = ops;
    a.m1 = c.sh->n1 >> (lc - 1);
    a.m2 = c.sh->n2 >> (lc - 1);
    a.nlev = L - lc + 1;
    a.band_top = L + 1 - lc;
    a.apx_in = lc == 1 ? in : c.apx(lc - 1);
    a.apx_in_plane = lc == 1 ? c.N() : (int64_t)a.m1 * a.m2;
    a.apx_out = lc == 1 ? out : c.apx(lc - 1);
    a.apx_out_plane = a.apx_in_plane;
    a.beta_next = beta_next;
    a.kw = c.ts.kw;
    a.tM1 = c.ts.tM1;
    a.tM2 = c.ts.tM2;
    a.tail = c.tail;
    if (c.ts.nt > 0 && !c.tail) return PD_ERR_HIP;
    a.p = p;
    if (rv) {  // the reverse sweep's combine and mask (COARSE_REVCM)
        a.rv_vbar = rv->rv_vbar;
        a.rv_zbar = rv->rv_zbar;
        a.rv_zbarm = rv->rv_zbarm;
        a.rv_wbar = rv->rv_wbar;
        a.rv_b = rv->rv_b;
        a.rv_first = rv->rv_first;
        a.rv_di = rv->rv_di;
    }
    const int groups = p.joint ? 1 : c.sh->channels;
    PD_TRY_HIP(timed(PD_K_COARSE, lc, c.st, [&] { return launch_coarse<T>(a, groups, c.st); }));
    return PD_OK;
}

// Fine synthesis levels lc-1 .. 1 (their approximation input comes from the
// coarse kernel's output, or from the state when there is no coarse kernel).
template <typename T>
int synth_fine(const Ctx<T> &c, const T *zc, const T *zp, T beta, T *out, DevIter di = DevIter{nullptr, 0})
{
    const int L = c.sh->levels, n1 = c.sh->n1, n2 = c.sh->n2;
    auto args = [&](int lev) {
        SynthArgs<T> a;
        a.f = c.f;
        a.zc = zc;
        a.zp = zp;
        a.beta = beta;
        a.di = di;
        a.plane = c.N();
        a.pitch = n1;
        a.apx = lev == L ? nullptr : c.apx(lev);
        a.apx_plane = (int64_t)(n1 >> lev) * (n2 >> lev);
        a.out = lev == 1 ? out : c.apx(lev - 1);
        a.out_pitch = lev == 1 ? n1 : (n1 >> (lev - 1));
        a.out_plane = lev == 1 ? c.N() : (int64_t)(n1 >> (lev - 1)) * (n2 >> (lev - 1));
        a.M1c = n1 >> lev;
        a.M2c = n2 >> lev;
        return a;
    };
    int lev = c.lc - 1;
    if (lev >= 3 && g_synth2) {  // the three coarsest fine levels in one launch
        const SynthArgs<T> v = args(lev), u = args(lev - 1), d = args(lev - 2);
        PD_TRY_HIP(
            timed(PD_K_SYNTH3, lev - 2, c.st, [&] { return launch_synth3<T>(d, u, v, c.sh->channels, c.st); }));
        lev -= 3;
    } else if (lev >= 2 && g_synth2) {  // the two coarsest fine levels in one launch
        const SynthArgs<T> u = args(lev), d = args(lev - 1);
        PD_TRY_HIP(timed(PD_K_SYNTH2, lev - 1, c.st, [&] { return launch_synth2<T>(d, u, c.sh->channels, c.st); }));
        lev -= 2;
    }
    for (; lev >= 1; --lev) {
        const SynthArgs<T> a = args(lev);
        PD_TRY_HIP(timed(PD_K_SYNTH, lev, c.st, [&] { return launch_synth<T>(a, c.sh->channels, c.st); }));
    }
    return PD_OK;
}

// x = Psi y, y = zc + beta (zc - zp): coarse kernel (synthesis only) + fine levels
template <typename T>
int synth_chain(const Ctx<T> &c, const T *zc, const T *zp, T beta, T *out, DevIter di = DevIter{nullptr, 0})
{
    int rc;
    if (c.lc <= c.sh->levels) {
        ProxArgs<T> p = prox_args<T>(c, zc, zp, nullptr, beta, T(0), nullptr, nullptr);
        p.di = di;
        if ((rc = coarse_step<T>(c, COARSE_SYN, nullptr, out, p, T(0))) != PD_OK) return rc;
    }
    return synth_fine<T>(c, zc, zp, beta, out, di);
}

// Fine analysis levels 1 .. lc-1: plain coefficients (MODE_PLAIN) or the fused
// gradient step + prox + momentum (MODE_PROX).
constexpr int64_t ANA2_MAX_INPUT = 512 * 512;

template <typename T>
int analysis_fine(const Ctx<T> &c, const T *in, int mode, const ProxArgs<T> &p)
{
    const int L = c.sh->levels, n1 = c.sh->n1, n2 = c.sh->n2;
    auto args = [&](int lev) {
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
        a.band_detail = L + 1 - lev;
        a.p = p;
        return a;
    };
    // Levels in pairs (one launch each) from the coarsest fine level down,
    // while the finer level of the pair reads at most ANA2_MAX_INPUT values per
    // channel (the latency-bound sizes; on larger planes the pair's overlapping
    // input regions cost more than the launch it saves); the rest one by one.
    int single = c.lc - 1;
    if (g_synth2 && !p.joint)
        while (single >= 2 && (int64_t)(n1 >> (single - 2)) * (n2 >> (single - 2)) <= ANA2_MAX_INPUT) single -= 2;
    for (int lev = 1; lev <= single; ++lev) {
        const AnalysisArgs<T> a = args(lev);
        PD_TRY_HIP(timed(PD_K_ANALYSIS, lev, c.st, [&] { return launch_analysis<T>(a, c.st); }));
    }
    for (int lev = single + 1; lev + 1 <= c.lc - 1; lev += 2) {
        const AnalysisArgs<T> a = args(lev), e = args(lev + 1);
        PD_TRY_HIP(timed(PD_K_ANALYSIS2, lev, c.st, [&] { return launch_analysis2<T>(a, e, c.st); }));
    }
    return PD_OK;
}

// Plain forward transform out = Psi^* in.
template <typename T>
int analysis_plain(const Ctx<T> &c, const T *in, T *out)
{
    int rc;
    ProxArgs<T> p = prox_args<T>(c, nullptr, nullptr, out, T(0), T(0), nullptr, nullptr);
    if ((rc = analysis_fine<T>(c, in, MODE_PLAIN, p)) != PD_OK) return rc;
    if (c.lc <= c.sh->levels) return coarse_step<T>(c, COARSE_ANA, in, nullptr, p, T(0));
    return PD_OK;
}

template <typename T>
int blur_step(const Ctx<T> &c, const pd_operator *op, const T *x, const T *f0, T *s, double *slots,
              T *racc = nullptr, T rscale = T(0))
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
    a.slots = slots;
    a.racc = racc;
    a.rscale = rscale;
    a.r = c.btab ? (T *)(c.ws + c.lay.r) : nullptr;
    a.tabs = c.btab;
    a.rows = 0;
    if (op->kind == PD_OP_PC) {  // product-convolution expansion (no reverse-mode accumulation)
        if (racc) return PD_ERR_UNSUPPORTED;
        PcArgs<T> p{x, f0, s, (const T *)op->taps, (const T *)op->mult, c.sh->n1, c.sh->n2, c.sh->channels,
                    op->radius, op->terms, c.N(), slots};
        PD_TRY_HIP(timed(PD_K_BLUR, 0, c.st, [&] { return launch_pcblur<T>(p, c.st); }));
        return PD_OK;
    }
    PD_TRY_HIP(timed(PD_K_BLUR, 0, c.st, [&] { return launch_blur<T>(a, op->kind == PD_OP_IDENTITY, c.st); }));
    return PD_OK;
}

// Fills the per-row profile tables of the two-kernel blur (row blur only);
// stream-ordered before the iterations that read them.
template <typename T>
int prep_blur(Ctx<T> &c, const pd_operator *op)
{
    if (op->kind != PD_OP_ROWBLUR) return PD_OK;
    T *tab = (T *)(c.ws + c.lay.btab);
    PD_TRY_HIP(launch_blur_tables<T>((const T *)op->taps, c.sh->n2, op->radius, tab, c.st));
    c.btab = tab;
    return PD_OK;
}

template <typename T>
Ctx<T> make_ctx(const pd_shape *sh, const pd_wavelet *wav, void *workspace, hipStream_t st, int joint)
{
    Ctx<T> c;
    c.sh = sh;
    c.f = make_filt<T>(wav);
    c.ws = (char *)workspace;
    c.lay = layout(sh, sizeof(T));
    c.st = st;
    c.lc = coarse_level<T>(sh, joint);
    c.tail = nullptr;
    c.ts = TailShape{0, 0, 0, 0};
    if (c.lc <= sh->levels) {
        c.ts = tail_shape(sh->n1 >> (c.lc - 1), sh->n2 >> (c.lc - 1), sh->levels - c.lc + 1);
        if (c.ts.nt > 0 && workspace) {
            const std::vector<T> &m = tail_matrices<T>(c.ts, wav);
            T *dst = (T *)(c.ws + c.lay.tail);
            if (hipMemcpyAsync(dst, m.data(), m.size() * sizeof(T), hipMemcpyHostToDevice, st) == hipSuccess)
                c.tail = dst;
        }
    }
    return c;
}

// Momentum of y(i) = z(i-1) + b (z(i-1) - z(i-2)):  b_{i-1} = (i-2)/(i+1), 0 for i = 1.
inline double beta_y(int i) { return i >= 2 ? (double)(i - 2) / (double)(i + 1) : 0.0; }

// One iteration (local index it, global i = i_first + it) of the recursion
// from (zc, zp) = (z(i-1), z(i-2)); z(i) is written in place of z(i-2).
// With di.it_dev set the launches take i from device memory (*it_dev +
// di.it_off == i), so that a captured graph of them replays for any i.
template <typename T>
int one_iteration(const Ctx<T> &c, const pd_operator *op, const pd_weights *w, T tau, const T *f0, const T *zc,
                  T *zp, int it, int i, int count, double *stats, int i_first, DevIter di, T *zsave = nullptr)
{
    const pd_shape *sh = c.sh;
    const hipStream_t st = c.st;
    const bool coarse = c.lc <= sh->levels;
    const T beta = (T)beta_y(i);
    const bool last = it == count - 1;
    double *sti = stats ? c.slots(it) : nullptr;
    int rc;
    // x = Psi y(i); the coarse part was produced by the previous iteration's coarse kernel
    if (it == 0) {
        if ((rc = synth_chain<T>(c, zc, zp, beta, c.x(), di)) != PD_OK) return rc;
    } else if ((rc = synth_fine<T>(c, zc, zp, beta, c.x(), di)) != PD_OK) {
        return rc;
    }
    if ((rc = blur_step<T>(c, op, c.x(), f0, c.s(), sti)) != PD_OK) return rc;
    // z(i) overwrites z(i-2) in place (each coefficient is read, then written, by one thread)
    ProxArgs<T> p = prox_args<T>(c, zc, zp, zp, beta, tau, w, sti);
    p.di = di;
    p.zsave = zsave;  // every coefficient of z(i) is stored by exactly one prox epilogue
    if (p.joint && sh->channels > 1) {
        // joint prox over several channels: per-channel plain analysis (fine levels, then the coarse
        // block) into the x plane (free after the blur), the joint prox over the whole plane, then
        // per-channel coarse synthesis of y(i+1) from (z(i), z(i-1)) -- the fused kernels' formulas
        ProxArgs<T> pa = prox_args<T>(c, nullptr, nullptr, c.x(), T(0), T(0), nullptr, nullptr);
        if ((rc = analysis_fine<T>(c, c.s(), MODE_PLAIN, pa)) != PD_OK) return rc;
        if (coarse && (rc = coarse_step<T>(c, COARSE_ANA, c.s(), nullptr, pa, T(0))) != PD_OK) return rc;
        JProxArgs<T> ja;
        ja.g = c.x();
        ja.m1 = sh->n1;
        ja.m2 = sh->n2;
        ja.nlev = sh->levels;
        ja.band_top = sh->levels;
        ja.p = p;
        PD_TRY_HIP(timed(PD_K_JPROX, 0, st, [&] { return launch_jprox<T>(ja, sh->channels, st); }));
        if (coarse && !last) {
            // y(i+1) = z(i) + b_i (z(i) - z(i-1)): z(i) is in zp (in place of z(i-2)), z(i-1) in zc
            ProxArgs<T> ps = prox_args<T>(c, zp, zc, nullptr, (T)beta_y(i + 1), T(0), nullptr, nullptr);
            ps.di = di;
            if (di.it_dev) ps.di.it_off = di.it_off + 1;  // the device iteration's beta of i + 1
            if ((rc = coarse_step<T>(c, COARSE_SYN, nullptr, c.x(), ps, T(0))) != PD_OK) return rc;
        }
    } else {
        if ((rc = analysis_fine<T>(c, c.s(), MODE_PROX, p)) != PD_OK) return rc;
        if (coarse) {
            const int ops = COARSE_ANA | COARSE_PROX | (last ? 0 : COARSE_SYN);
            if ((rc = coarse_step<T>(c, ops, c.s(), c.x(), p, (T)beta_y(i + 1))) != PD_OK) return rc;
        }
    }
    if (stats && ((it + 1) % PD_RING == 0 || last)) {  // fold the ring into stats
        const int cnt = (it % PD_RING) + 1, it0 = it + 1 - cnt;
        if (di.it_dev) {  // it0 = (*it_dev + it_off - i_first) + 1 - cnt
            const int sub = i_first - di.it_off - 1 + cnt;
            PD_TRY_HIP(launch_stats_finalize_dev(c.ring(), stats, di.it_dev, sub, cnt, st));
        } else {
            PD_TRY_HIP(timed(PD_K_OTHER, 0, st, [&] { return launch_stats_finalize(c.ring(), stats, it0, cnt, st); }));
        }
    }
    return PD_OK;
}

// ---------------------------------------------------- graph replay ---
// The middle iterations (neither the first nor the last) run in chunks of
// PD_RING starting at local index 1 mod PD_RING: the launches of a chunk are
// captured once into a HIP graph whose kernels read the iteration number
// from device memory, and that executable graph is replayed for every chunk
// of this and of later solves with the same arguments (a small cache keyed
// by everything the launches bake in).  Each replay is preceded by a one-
// thread kernel that stores the chunk's first iteration number.
bool g_graphs = true;
struct CachedGraph {
    std::vector<char> key;
    hipGraphExec_t exec;
    hipEvent_t done;  // recorded after every launch of exec
};
std::vector<CachedGraph> g_graph_cache;  // least recently used first
std::vector<CachedGraph> g_graph_retired;  // evicted, destroyed once their last launch completed

void sweep_retired()
{
    for (size_t k = 0; k < g_graph_retired.size();) {
        if (hipEventQuery(g_graph_retired[k].done) == hipSuccess) {
            (void)hipGraphExecDestroy(g_graph_retired[k].exec);
            (void)hipEventDestroy(g_graph_retired[k].done);
            g_graph_retired.erase(g_graph_retired.begin() + k);
        } else {
            ++k;
        }
    }
    (void)hipGetLastError();
}
std::mutex g_graph_mu;
constexpr size_t GRAPH_CACHE = 32;

template <typename V>
void key_put(std::vector<char> &k, const V &v)
{
    const char *p = (const char *)&v;
    k.insert(k.end(), p, p + sizeof(V));
}

hipStream_t capture_stream(int dev)
{
    static std::map<int, hipStream_t> streams;  // guarded by g_graph_mu
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = s;
    return s;
}

// Looks up the executable graph cached under `key`, or, if allowed, captures
// one by running record(capture_stream) and caches it; then stores `it_value`
// in *it_dev, replays the graph on st and records its completion event, all
// under the cache lock (no other thread can retire and destroy the graph
// between the lookup and the record).  Returns false when there is no graph
// (the caller runs the work eagerly) and sets *err on a HIP error.
template <typename F>
bool replay_graph(const std::vector<char> &key, bool may_capture, F &&record, int *it_dev, int it_value,
                  hipStream_t st, int *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lock(g_graph_mu);
    sweep_retired();
    hipGraphExec_t ex = nullptr;
    hipEvent_t done = nullptr;
    for (size_t k = 0; k < g_graph_cache.size(); ++k)
        if (g_graph_cache[k].key == key) {
            CachedGraph e = g_graph_cache[k];
            g_graph_cache.erase(g_graph_cache.begin() + k);
            g_graph_cache.push_back(e);
            ex = e.exec;
            done = e.done;
            break;
        }
    if (!ex) {
        if (!may_capture) return false;
        hipStream_t cs = capture_stream(dev);
        if (!cs) return false;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        const int rc = record(cs);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc == PD_OK && e == hipSuccess && g && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess)
            ex = nullptr;
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (!ex) return false;
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGraphExecDestroy(ex);
            (void)hipGetLastError();
            return false;
        }
        if (g_graph_cache.size() >= GRAPH_CACHE) {  // it may still be queued: retire, destroy later
            g_graph_retired.push_back(g_graph_cache.front());
            g_graph_cache.erase(g_graph_cache.begin());
        }
        g_graph_cache.push_back(CachedGraph{key, ex, done});
    }
    if (launch_set_int(it_dev, it_value, st) != hipSuccess || hipGraphLaunch(ex, st) != hipSuccess ||
        hipEventRecord(done, st) != hipSuccess)
        *err = PD_ERR_HIP;
    return true;
}

// Replays (capturing first if allowed) the chunk of PD_RING iterations that
// starts at local index it_a.  The key holds everything the launches bake in.
template <typename T>
bool launch_chunk_graph(const Ctx<T> &c, const pd_operator *op, const pd_weights *w, T tau, const T *f0, T *zc,
                        T *zp, int it_a, int count, double *stats, int i_first, bool may_capture, int *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::vector<char> key;
    key_put(key, 'S');
    key_put(key, (int)sizeof(T));
    key_put(key, dev);
    key_put(key, *c.sh);
    key_put(key, c.ws);
    key_put(key, c.lc);
    key_put(key, c.tail);
    key_put(key, c.f);
    key_put(key, op->kind);
    key_put(key, op->radius);
    key_put(key, op->taps);
    key_put(key, op->terms);
    key_put(key, op->mult);
    key_put(key, w->coeff_w);
    key_put(key, w->joint);
    for (int k = 0; k <= c.sh->levels; ++k) key_put(key, w->level_w ? w->level_w[k] : 0.0);
    key_put(key, tau);
    key_put(key, f0);
    key_put(key, zc);
    key_put(key, zp);
    key_put(key, stats);
    key_put(key, i_first);
    auto record = [&](hipStream_t cs) -> int {
        Ctx<T> cc = c;
        cc.st = cs;
        int rc = PD_OK;
        T *a = zc, *b = zp;
        for (int j = 0; j < PD_RING && rc == PD_OK; ++j) {
            rc = one_iteration<T>(cc, op, w, tau, f0, a, b, it_a + j, i_first + it_a + j, count, stats, i_first,
                                  DevIter{c.it_dev(), j});
            std::swap(a, b);
        }
        return rc;
    };
    return replay_graph(key, may_capture, record, c.it_dev(), i_first + it_a, c.st, err);
}

// Iterations i = i_first .. i_first+count-1 of the recursion from the state
// (zc, zp) = (z(i_first-1), z(i_first-2)); on return the pointers hold
// (z(last), z(last-1)).  z(i) is written in place of z(i-2).  stats (nullable)
// receives 3 doubles per iteration; seg (nullable) receives a copy of every
// z(i) (count planes), for the reverse sweep.
template <typename T>
int iterate(const Ctx<T> &c, const pd_operator *op, const pd_weights *w, T tau, const T *f0, T *&zc, T *&zp,
            int i_first, int count, double *stats, T *seg)
{
    const hipStream_t st = c.st;
    const int64_t NC = c.N() * c.sh->channels;
    const bool graphs = g_graphs && !g_timing && !seg && !c.eager;
    int rc;
    if (stats && count > 0) PD_TRY_HIP(launch_fill<double>(c.ring(), 0.0, (int64_t)PD_RING * 3 * PD_NSLOT, st));
    // capturing pays off only when the graph is replayed several times
    int chunks = 0;
    for (int it = 1; it + PD_RING < count; it += PD_RING) ++chunks;
    const bool may_capture = chunks >= 4;
    for (int it = 0; it < count;) {
        if (graphs && !seg && it % PD_RING == 1 && it + PD_RING < count) {
            int err = PD_OK;
            if (launch_chunk_graph<T>(c, op, w, tau, f0, zc, zp, it, count, stats, i_first, may_capture, &err)) {
                if (err != PD_OK) return err;
                it += PD_RING;  // an even number of swaps: (zc, zp) unchanged
                continue;
            }
        }
        if ((rc = one_iteration<T>(c, op, w, tau, f0, zc, zp, it, i_first + it, count, stats, i_first,
                                   DevIter{nullptr, 0}, seg ? seg + (int64_t)it * NC : nullptr)) != PD_OK)
            return rc;
        T *t = zc;
        zc = zp;
        zp = t;
        ++it;
    }
    return PD_OK;
}

// The recomputation of pd_backward: count iterations from (zc, zp), every
// z(i) also stored in seg by the kernels that compute it.  it_dev set: the launches read i = *it_dev +
// local index from device memory (for a captured segment).
template <typename T>
int iterate_seg(const Ctx<T> &c, const pd_operator *op, const pd_weights *w, T tau, const T *f0, T *zc, T *zp,
                int i_first, int count, T *seg, const int *it_dev)
{
    const int64_t NC = c.N() * c.sh->channels;
    int rc;
    for (int it = 0; it < count; ++it) {
        if ((rc = one_iteration<T>(c, op, w, tau, f0, zc, zp, it, i_first + it, count, nullptr, i_first,
                                   DevIter{it_dev, it_dev ? it : 0}, seg + (int64_t)it * NC)) != PD_OK)
            return rc;
        std::swap(zc, zp);
    }
    return PD_OK;
}

template <typename T>
int solve_impl(const pd_shape *sh, const pd_operator *op, const pd_wavelet *wav, const pd_weights *w,
               const pd_params *prm, const T *f0, T *z_cur, T *z_prev, int init, T *f_out,
               double *stats, void *workspace, size_t ws_bytes, hipStream_t st, bool eager = false)
{
    // size check before make_ctx, which queues the tail-matrix upload into the workspace
    if (ws_bytes < layout(sh, sizeof(T)).total) return PD_ERR_WORKSPACE;
    Ctx<T> c = make_ctx<T>(sh, wav, workspace, st, w->joint);
    c.eager = eager;
    const int64_t NC = c.N() * sh->channels;
    int rc;
    if ((rc = prep_blur<T>(c, op)) != PD_OK) return rc;
    if (init) {
        if ((rc = analysis_plain<T>(c, f0, z_cur)) != PD_OK) return rc;
        PD_TRY_HIP(timed(PD_K_OTHER, 0, st, [&] { return launch_copy<T>(z_cur, z_prev, NC, st); }));
    }
    if (prm->check_finite) PD_TRY_HIP(launch_set_int(c.flag(), 0, st));  // a kernel, not a memset node
    T *zc = z_cur, *zp = z_prev;
    if ((rc = iterate<T>(c, op, w, (T)prm->tau, f0, zc, zp, prm->iter_offset + 1, prm->iters, stats, nullptr)) != PD_OK)
        return rc;
    if (zc != z_cur) {  // odd number of iterations: swap the two planes
        T *tmp = c.x();
        PD_TRY_HIP(timed(PD_K_OTHER, 0, st, [&] { return launch_copy<T>(z_cur, tmp, NC, st); }));
        PD_TRY_HIP(timed(PD_K_OTHER, 0, st, [&] { return launch_copy<T>(z_prev, z_cur, NC, st); }));
        PD_TRY_HIP(timed(PD_K_OTHER, 0, st, [&] { return launch_copy<T>(tmp, z_prev, NC, st); }));
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

// ---------------------------------------------------------------- batched --
// Lock-step solve of many images of uneven sizes: every phase of an iteration
// (coarse synthesis, fine synthesis level l, blur, fine analysis level l,
// coarse analysis + prox) is ONE launch over the tiles of all images that
// have that phase.  Per-image argument blocks live in device tables built
// once per call; the momentum, the buffer parity and the iteration index are
// passed by value each iteration.  Same tile code and arithmetic as pd_solve.

struct BImg {
    pd_shape sh;
    int lc;
    int64_t off;          // element offset in the packed image arrays
    size_t apx[PD_MAXL + 1];
    size_t slots;
    bool split;           // the blur as the two marching kernels (row blur, wide enough)
    size_t btab;          // their per-row profile tables
};

struct BLayout {
    std::vector<BImg> img;
    int64_t total;        // packed elements
    size_t zA, zB, x, s, r, flag, it, tab, tab_bytes, total_bytes;
    int maxfine;
};

// Images at least this wide run the batched blur as the two marching kernels
// (strips of 128 columns, blocks of BATCH_SPLIT_ROWS rows per wave); narrower
// ones as the 32-row tile kernel.  The same sums either way.  Measured on the
// 64-image batch (sides 96..1024): the batch's blur takes 283 us per iteration
// with the tile kernel alone, 167 us with the marching pair from 256 columns
// and 39-row blocks, 147 us from 128 columns and 58-row blocks.
constexpr int BATCH_SPLIT_MIN_N1 = 128;
constexpr int BATCH_SPLIT_ROWS = 58;

template <typename Args>
struct Table {
    std::vector<Args> args;
    std::vector<int> start{0};
    size_t off = 0;       // byte offset of args in the table region; start follows
    void add(const Args &a, int tiles)
    {
        args.push_back(a);
        start.push_back(start.back() + tiles);
    }
    int n() const { return (int)args.size(); }
    int tiles() const { return start.back(); }
};

size_t table_bytes_upper(int batch, int maxl)
{
    // per image at most: 2 coarse SYN + 2 coarse PROX + init coarse + 3 blur;
    // per level synth (iteration and final) + analysis (plain, prox), all < 1 KiB
    return align_up((size_t)batch * (10 + 4 * (size_t)maxl) * 1024 + 64 * 1024);
}

template <typename T>
BLayout batched_layout(int batch, const pd_image_desc *d)
{
    BLayout L;
    L.total = 0;
    L.maxfine = 0;
    int maxl = 0;
    for (int b = 0; b < batch; ++b) {
        BImg im;
        im.sh = d[b].shape;
        im.lc = coarse_level<T>(&im.sh, d[b].w.joint);
        im.off = L.total;
        im.split = d[b].op.kind == PD_OP_ROWBLUR && im.sh.n1 >= BATCH_SPLIT_MIN_N1;
        im.btab = 0;
        L.total += (int64_t)im.sh.n1 * im.sh.n2 * im.sh.channels;
        L.maxfine = std::max(L.maxfine, im.lc - 1);
        maxl = std::max(maxl, (int)im.sh.levels);
        L.img.push_back(im);
    }
    const size_t es = sizeof(T), plane = align_up(es * L.total);
    size_t off = 0;
    L.zA = off;
    off += plane;
    L.zB = off;
    off += plane;
    L.x = off;
    off += plane;
    L.s = off;
    off += plane;
    L.r = off;  // r = H x - f0 of the marching blur
    off += plane;
    for (auto &im : L.img) {
        for (int j = 0; j <= PD_MAXL; ++j) im.apx[j] = 0;
        for (int j = 1; j < im.sh.levels; ++j) {
            im.apx[j] = off;
            off = align_up(off + es * im.sh.channels * (size_t)(im.sh.n1 >> j) * (im.sh.n2 >> j));
        }
        im.slots = off;
        off = align_up(off + (size_t)PD_RING * 3 * PD_NSLOT * sizeof(double));
        if (im.split) {
            im.btab = off;
            off = align_up(off + 2 * (size_t)im.sh.n2 * BLUR_TAB_PITCH * es);
        }
    }
    L.flag = off;
    off = align_up(off + 256);
    L.it = off;  // device iteration number of replayed graphs
    off = align_up(off + 256);
    L.tab = off;
    L.tab_bytes = table_bytes_upper(batch, maxl);
    off += L.tab_bytes;
    L.total_bytes = off;
    return L;
}

// Pinned host staging for the descriptor tables: the upload is asynchronous
// and a buffer is reused only after the event recorded behind its last copy
// has completed, so the call never waits for the device.
struct Staging {
    void *host;
    size_t bytes;
    hipEvent_t done;
};
std::mutex g_stage_mu;
std::vector<Staging> g_stage;

int upload_async(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Staging *use = nullptr;
    for (auto &e : g_stage)
        if (e.bytes >= bytes && hipEventQuery(e.done) == hipSuccess) {
            use = &e;
            break;
        }
    (void)hipGetLastError();  // a pending event reports hipErrorNotReady
    if (!use) {
        Staging e{nullptr, std::max(bytes, (size_t)1 << 16), nullptr};
        if (hipHostMalloc(&e.host, e.bytes, hipHostMallocDefault) != hipSuccess) return PD_ERR_HIP;
        if (hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(e.host);
            return PD_ERR_HIP;
        }
        g_stage.push_back(e);
        use = &g_stage.back();
    }
    std::memcpy(use->host, src, bytes);
    PD_TRY_HIP(hipMemcpyAsync(dst, use->host, bytes, hipMemcpyHostToDevice, st));
    PD_TRY_HIP(hipEventRecord(use->done, st));
    return PD_OK;
}

template <typename T>
int solve_batched_impl(int batch, const pd_image_desc *d, const pd_wavelet *wav, int iters, const T *f0p,
                       T *fop, double *stats, void *workspace, size_t ws_bytes, hipStream_t st)
{
    BLayout L = batched_layout<T>(batch, d);
    if (ws_bytes < L.total_bytes) return PD_ERR_WORKSPACE;
    char *ws = (char *)workspace;
    const Filt<T> f = make_filt<T>(wav);
    T *zA = (T *)(ws + L.zA), *zB = (T *)(ws + L.zB), *X = (T *)(ws + L.x), *S = (T *)(ws + L.s);
    T *Rp = (T *)(ws + L.r);
    int *flag = (int *)(ws + L.flag);
    int *it_dev = (int *)(ws + L.it);
    // joint prox: every image has the same channel count (checked by the caller)
    const int nch = d[0].w.joint ? d[0].shape.channels : 0;

    // tables: init (plain analysis, coarse plain), iteration (coarse syn, synth,
    // blur, analysis, coarse prox[+syn]), final synthesis into f_out
    const int MF = L.maxfine;
    std::vector<Table<AnalysisArgs<T>>> t_init_ana(MF + 1), t_ana(MF + 1);
    std::vector<Table<SynthArgs<T>>> t_syn(MF + 1), t_fsyn(MF + 1);
    Table<CoarseArgs<T>> t_init_co, t_cosyn, t_fcosyn, t_coprox_syn, t_coprox;
    Table<BlurArgs<T>> t_blur, t_blur_h, t_blur_ht;  // tile kernel; the marching pair (same args)
    std::vector<double *> slots_tab(batch), stats_tab(batch);
    const T *f_zfinal = (iters % 2 == 0) ? zA : zB;  // z(K) after K in-place iterations
    // host image of the table region: tail matrices first (deduplicated), then the tables
    std::vector<char> host;
    std::map<std::vector<int>, size_t> tail_off;

    for (int b = 0; b < batch; ++b) {
        const BImg &im = L.img[b];
        const pd_shape *sh = &im.sh;
        Ctx<T> c;
        c.sh = sh;
        c.f = f;
        c.ws = ws;
        c.st = st;
        c.lc = im.lc;
        c.lay.x = c.lay.s = c.lay.flag = 0;
        c.lay.slots = im.slots;
        for (int j = 0; j <= PD_MAXL; ++j) c.lay.apx[j] = im.apx[j];
        const int64_t N = (int64_t)sh->n1 * sh->n2;
        const int n1 = sh->n1, n2 = sh->n2, Lv = sh->levels, C = sh->channels;
        const int groups = nch ? 1 : C;  // tile sets / coarse workgroups per image
        double *slots = stats ? (double *)(ws + im.slots) : nullptr;
        double *stb = stats ? stats + (size_t)b * iters * 3 : nullptr;
        slots_tab[b] = slots;
        stats_tab[b] = stb;
        const pd_weights &w = d[b].w;
        T *zAb = zA + im.off, *zBb = zB + im.off, *Xb = X + im.off, *Sb = S + im.off;
        const T *F0b = f0p + im.off;
        T *FOb = fop + im.off;
        ProxArgs<T> pp = prox_args<T>(c, zAb, zBb, zBb, T(0), (T)d[b].tau, &w, slots);
        pp.flag = flag;
        ProxArgs<T> pplain = prox_args<T>(c, nullptr, nullptr, zAb, T(0), T(0), nullptr, nullptr);
        pplain.flag = flag;
        pplain.joint = pp.joint;  // same tile grouping in the plain transform
        const bool coarse = im.lc <= Lv;
        // fine levels
        for (int lev = 1; lev <= im.lc - 1; ++lev) {
            AnalysisArgs<T> a;
            a.f = f;
            a.in = lev == 1 ? Sb : c.apx(lev - 1);
            a.in_pitch = lev == 1 ? n1 : (n1 >> (lev - 1));
            a.in_plane = lev == 1 ? N : (int64_t)(n1 >> (lev - 1)) * (n2 >> (lev - 1));
            a.M1c = n1 >> lev;
            a.M2c = n2 >> lev;
            a.last = lev == Lv;
            a.apx_out = lev < Lv ? c.apx(lev) : nullptr;
            a.apx_plane = (int64_t)(n1 >> lev) * (n2 >> lev);
            a.band_detail = Lv + 1 - lev;
            tiles_analysis(a.M1c, a.M2c, &a.tx, &a.ty);
            const int tiles = a.tx * a.ty * groups;
            a.mode = MODE_PROX;
            a.p = pp;
            t_ana[lev].add(a, tiles);
            a.mode = MODE_PLAIN;
            a.p = pplain;
            if (lev == 1) a.in = F0b;
            t_init_ana[lev].add(a, tiles);

            SynthArgs<T> sa;
            sa.di = DevIter{nullptr, 0};
            sa.f = f;
            sa.zc = zAb;
            sa.zp = zBb;
            sa.beta = T(0);
            sa.plane = N;
            sa.pitch = n1;
            sa.apx = lev == Lv ? nullptr : c.apx(lev);
            sa.apx_plane = (int64_t)(n1 >> lev) * (n2 >> lev);
            sa.out = lev == 1 ? Xb : c.apx(lev - 1);
            sa.out_pitch = lev == 1 ? n1 : (n1 >> (lev - 1));
            sa.out_plane = lev == 1 ? N : (int64_t)(n1 >> (lev - 1)) * (n2 >> (lev - 1));
            sa.M1c = n1 >> lev;
            sa.M2c = n2 >> lev;
            tiles_synth(sa.M1c, sa.M2c, &sa.tx, &sa.ty);
            t_syn[lev].add(sa, sa.tx * sa.ty * C);
            sa.zc = sa.zp = f_zfinal + im.off;
            if (lev == 1) sa.out = FOb;
            t_fsyn[lev].add(sa, sa.tx * sa.ty * C);
        }
        BlurArgs<T> ba;
        ba.x = Xb;
        ba.f0 = F0b;
        ba.s = Sb;
        ba.taps = (const T *)d[b].op.taps;
        ba.n1 = n1;
        ba.n2 = n2;
        ba.C = C;
        ba.R = d[b].op.radius;
        ba.plane = N;
        ba.slots = slots;
        ba.racc = nullptr;
        ba.rscale = T(0);
        ba.r = Rp + im.off;
        ba.tabs = im.split ? (const T *)(ws + im.btab) : nullptr;
        ba.rows = im.split ? BATCH_SPLIT_ROWS : 0;
        if (im.split) {  // tx, ty = workgroups per channel of the r and H^T kernels
            tiles_blur_split(n1, n2, BATCH_SPLIT_ROWS, &ba.tx, &ba.ty);
            t_blur_h.add(ba, ba.tx * C);
            t_blur_ht.add(ba, ba.ty * C);
        } else {
            tiles_blur(n1, n2, &ba.tx, &ba.ty, 32);
            t_blur.add(ba, ba.tx * ba.ty * C);
        }
        if (coarse) {
            CoarseArgs<T> ca;
            ca.f = f;
            ca.m1 = n1 >> (im.lc - 1);
            ca.m2 = n2 >> (im.lc - 1);
            ca.nlev = Lv - im.lc + 1;
            ca.band_top = Lv + 1 - im.lc;
            ca.apx_in = im.lc == 1 ? Sb : c.apx(im.lc - 1);
            ca.apx_in_plane = im.lc == 1 ? N : (int64_t)ca.m1 * ca.m2;
            ca.apx_out = im.lc == 1 ? Xb : c.apx(im.lc - 1);
            ca.apx_out_plane = ca.apx_in_plane;
            ca.beta_next = T(0);
            const TailShape ts = tail_shape(ca.m1, ca.m2, ca.nlev);
            ca.kw = ts.kw;
            ca.tM1 = ts.tM1;
            ca.tM2 = ts.tM2;
            ca.tail = nullptr;
            if (ts.nt > 0) {
                std::vector<int> key{ts.tM1, ts.tM2, ts.nt};
                auto itk = tail_off.find(key);
                size_t o;
                if (itk == tail_off.end()) {
                    const std::vector<T> &m = tail_matrices<T>(ts, wav);
                    o = align_up(host.size());
                    host.resize(o + m.size() * sizeof(T));
                    std::memcpy(host.data() + o, m.data(), m.size() * sizeof(T));
                    tail_off[key] = o;
                } else {
                    o = itk->second;
                }
                ca.tail = (const T *)(ws + L.tab + o);
            }
            ca.ops = COARSE_ANA | COARSE_PROX | COARSE_SYN;
            ca.p = pp;
            t_coprox_syn.add(ca, groups);
            ca.ops = COARSE_ANA | COARSE_PROX;
            t_coprox.add(ca, groups);
            ca.ops = COARSE_SYN;
            t_cosyn.add(ca, groups);
            ca.p.zc = ca.p.zp = f_zfinal + im.off;
            if (im.lc == 1) ca.apx_out = FOb;
            t_fcosyn.add(ca, groups);
            ca.ops = COARSE_ANA;
            ca.p = pplain;
            if (im.lc == 1) ca.apx_in = F0b;
            ca.apx_out = nullptr;
            t_init_co.add(ca, groups);
        }
    }

    // upload every table into the workspace table region
    auto place = [&](auto &t) {
        if (t.n() == 0) return;
        using A = typename std::decay_t<decltype(t.args)>::value_type;
        size_t o = align_up(host.size());
        t.off = o;
        size_t sa = t.args.size() * sizeof(A);
        size_t ss = t.start.size() * sizeof(int);
        host.resize(align_up(o + sa) + ss);
        std::memcpy(host.data() + o, t.args.data(), sa);
        std::memcpy(host.data() + align_up(o + sa), t.start.data(), ss);
    };
    for (auto &t : t_init_ana) place(t);
    for (auto &t : t_ana) place(t);
    for (auto &t : t_syn) place(t);
    for (auto &t : t_fsyn) place(t);
    place(t_init_co);
    place(t_cosyn);
    place(t_fcosyn);
    place(t_coprox_syn);
    place(t_coprox);
    place(t_blur);
    place(t_blur_h);
    place(t_blur_ht);
    size_t o_sl = align_up(host.size());
    host.resize(o_sl + batch * sizeof(double *));
    std::memcpy(host.data() + o_sl, slots_tab.data(), batch * sizeof(double *));
    size_t o_st = align_up(host.size());
    host.resize(o_st + batch * sizeof(double *));
    std::memcpy(host.data() + o_st, stats_tab.data(), batch * sizeof(double *));
    if (host.size() > L.tab_bytes) return PD_ERR_UNSUPPORTED;
    char *tab = ws + L.tab;
    int rc;
    if ((rc = upload_async(tab, host.data(), host.size(), st)) != PD_OK) return rc;
    for (int b = 0; b < batch; ++b)  // the marching blur's profile tables, before the first iteration
        if (L.img[b].split)
            PD_TRY_HIP(launch_blur_tables<T>((const T *)d[b].op.taps, L.img[b].sh.n2, d[b].op.radius,
                                             (T *)(ws + L.img[b].btab), st));

    auto targs = [&](auto &t) {
        using A = typename std::decay_t<decltype(t.args)>::value_type;
        return (const A *)(tab + t.off);
    };
    auto tstart = [&](auto &t) {
        using A = typename std::decay_t<decltype(t.args)>::value_type;
        return (const int *)(tab + align_up(t.off + t.args.size() * sizeof(A)));
    };
    size_t colds = 0;
    for (auto &im : L.img)
        if (im.lc <= im.sh.levels)
            colds = std::max(colds, coarse_lds_bytes<T>(im.sh.n1 >> (im.lc - 1), im.sh.n2 >> (im.lc - 1),
                                                        nch ? nch : 1));

    auto run_coarse = [&](Table<CoarseArgs<T>> &t, Dyn<T> dy, hipStream_t s) -> int {
        if (t.n() == 0) return PD_OK;
        PD_TRY_HIP(timed(PD_K_COARSE, 0, s, [&] {
            return launch_coarse_b<T>(targs(t), tstart(t), t.n(), t.tiles(), colds, nch, dy, s);
        }));
        return PD_OK;
    };
    auto run_synth = [&](std::vector<Table<SynthArgs<T>>> &ts, Dyn<T> dy, hipStream_t s) -> int {
        for (int lev = MF; lev >= 1; --lev) {
            auto &t = ts[lev];
            if (t.n() == 0) continue;
            PD_TRY_HIP(timed(PD_K_SYNTH, lev, s,
                             [&] { return launch_synth_b<T>(targs(t), tstart(t), t.n(), t.tiles(), dy, s); }));
        }
        return PD_OK;
    };
    auto run_ana = [&](std::vector<Table<AnalysisArgs<T>>> &ts, Dyn<T> dy, hipStream_t s) -> int {
        for (int lev = 1; lev <= MF; ++lev) {
            auto &t = ts[lev];
            if (t.n() == 0) continue;
            PD_TRY_HIP(timed(PD_K_ANALYSIS, lev, s, [&] {
                return launch_analysis_b<T>(targs(t), tstart(t), t.n(), t.tiles(), nch, dy, s);
            }));
        }
        return PD_OK;
    };
    // One iteration (local index it, i = it + 1).  dy carries the momenta, or
    // (replay) the device iteration number they are computed from; the stats
    // fold reads its first entry as it0 (+ *it_dev when replayed).
    auto one_it = [&](int it, Dyn<T> dy, int fold_it0, hipStream_t s) -> int {
        int r;
        if (it == 0 && (r = run_coarse(t_cosyn, dy, s)) != PD_OK) return r;
        if ((r = run_synth(t_syn, dy, s)) != PD_OK) return r;
        // one timed entry for the batch's whole blur (tile kernel and marching pair)
        PD_TRY_HIP(timed(PD_K_BLUR, 0, s, [&] {
            if (t_blur.n() > 0) {
                hipError_t e = launch_blur_b<T>(targs(t_blur), tstart(t_blur), t_blur.n(), t_blur.tiles(), dy.ring, s);
                if (e != hipSuccess) return e;
            }
            if (t_blur_h.n() > 0)
                return launch_blur_split_b<T>(targs(t_blur_h), tstart(t_blur_h), tstart(t_blur_ht), t_blur_h.n(),
                                              t_blur_h.tiles(), t_blur_ht.tiles(), BATCH_SPLIT_ROWS, dy.ring, s);
            return hipSuccess;
        }));
        if ((r = run_ana(t_ana, dy, s)) != PD_OK) return r;
        if ((r = run_coarse(it == iters - 1 ? t_coprox : t_coprox_syn, dy, s)) != PD_OK) return r;
        if (stats && ((it + 1) % PD_RING == 0 || it == iters - 1)) {
            const int cnt = (it % PD_RING) + 1;
            PD_TRY_HIP(launch_stats_finalize_b((double *const *)(tab + o_sl), (double *const *)(tab + o_st), batch,
                                               fold_it0, cnt, dy.it_dev, s));
        }
        return PD_OK;
    };

    Dyn<T> d0{T(0), T(0), 0, 0, nullptr, 0};
    // init: z(0) = Psi^* f0 into zA, copied to zB
    if ((rc = run_ana(t_init_ana, d0, st)) != PD_OK) return rc;
    if ((rc = run_coarse(t_init_co, d0, st)) != PD_OK) return rc;
    PD_TRY_HIP(launch_copy<T>(zA, zB, L.total, st));
    if (stats)
        for (int b = 0; b < batch; ++b)
            PD_TRY_HIP(launch_fill<double>(slots_tab[b], 0.0, (int64_t)PD_RING * 3 * PD_NSLOT, st));
    // the middle iterations run in replayed chunks of PD_RING (as pd_solve's)
    const bool graphs = g_graphs && !g_timing;
    int chunks = 0;
    for (int it = 1; it + PD_RING < iters; it += PD_RING) ++chunks;
    const bool may_capture = chunks >= 4;
    std::vector<char> key;
    if (graphs && chunks > 0) {
        int dev = 0;
        PD_TRY_HIP(hipGetDevice(&dev));
        key_put(key, 'B');
        key_put(key, (int)sizeof(T));
        key_put(key, dev);
        key_put(key, ws);
        key_put(key, f0p);
        key_put(key, stats);
        key_put(key, iters);
        key_put(key, batch);
        key_put(key, f);
        // the tables are rebuilt each call from these: equal bytes, equal launches
        const size_t h0 = key.size();
        key.resize(h0 + host.size());
        std::memcpy(key.data() + h0, host.data(), host.size());
    }
    for (int it = 0; it < iters;) {
        if (graphs && it % PD_RING == 1 && it + PD_RING < iters) {
            const int it_a = it;
            auto record = [&](hipStream_t cs) -> int {
                int r = PD_OK;
                for (int j = 0; j < PD_RING && r == PD_OK; ++j) {
                    const int itj = it_a + j;
                    const int cnt = (itj % PD_RING) + 1;
                    // i = *it_dev + j with *it_dev = it_a + 1; fold entries from (i - 1) + 1 - cnt
                    Dyn<T> dy{T(0), T(0), itj & 1, itj % PD_RING, it_dev, j};
                    r = one_it(itj, dy, j - cnt, cs);
                }
                return r;
            };
            int err = PD_OK;
            if (replay_graph(key, may_capture, record, it_dev, it_a + 1, st, &err)) {
                if (err != PD_OK) return err;
                it += PD_RING;
                continue;
            }
        }
        const int i = 1 + it;
        Dyn<T> dy{(T)beta_y(i), (T)beta_y(i + 1), it & 1, it % PD_RING, nullptr, 0};
        if ((rc = one_it(it, dy, it + 1 - ((it % PD_RING) + 1), st)) != PD_OK) return rc;
        ++it;
    }
    // f = Psi z(K)
    Dyn<T> dz{T(0), T(0), 0, 0, nullptr, 0};
    if ((rc = run_coarse(t_fcosyn, dz, st)) != PD_OK) return rc;
    if ((rc = run_synth(t_fsyn, dz, st)) != PD_OK) return rc;
    return PD_OK;
}

}  // namespace

extern "C" size_t pd_batched_workspace_size(int32_t batch, const pd_image_desc *descs, int32_t dtype)
{
    if (batch < 1 || !descs || check_dtype(dtype) != PD_OK) return 0;
    for (int b = 0; b < batch; ++b)
        if (check_shape(&descs[b].shape) != PD_OK) return 0;
    return dtype == PD_F64 ? batched_layout<double>(batch, descs).total_bytes
                           : batched_layout<float>(batch, descs).total_bytes;
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
        if ((rc = check_shape(&d.shape)) || (rc = check_op(&d.op, &d.shape)) || (rc = check_weights(&d.w, &d.shape)))
            return rc;
        if (d.op.kind != PD_OP_ROWBLUR) return PD_ERR_UNSUPPORTED;
        if (d.offset < 0) return PD_ERR_ARG;
        if (!std::isfinite(d.tau) || d.tau <= 0.0) return PD_ERR_TAU;
        // one launch per phase: every image takes the same prox kind (and, joint, channel count)
        if ((d.w.joint != 0) != (descs[0].w.joint != 0)) return PD_ERR_UNSUPPORTED;
        if (d.w.joint && d.shape.channels != descs[0].shape.channels) return PD_ERR_UNSUPPORTED;
    }
    // images must be packed back to back in order (offset = running sum)
    int64_t run = 0;
    for (int b = 0; b < batch; ++b) {
        if (descs[b].offset != run) return PD_ERR_ARG;
        run += (int64_t)descs[b].shape.n1 * descs[b].shape.n2 * descs[b].shape.channels;
    }
    if (ws_bytes < pd_batched_workspace_size(batch, descs, dtype)) return PD_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PD_F32)
        return solve_batched_impl<float>(batch, descs, wav, iters, (const float *)f0_packed, (float *)f_out_packed,
                                         stats, workspace, ws_bytes, st);
    return solve_batched_impl<double>(batch, descs, wav, iters, (const double *)f0_packed,
                                      (double *)f_out_packed, stats, workspace, ws_bytes, st);
}


extern "C" int pd_fuse_enable(int32_t enable)
{
    g_synth2 = enable != 0;
    return PD_OK;
}

extern "C" int pd_graphs_enable(int32_t enable)
{
    g_graphs = enable != 0;
    return PD_OK;
}

extern "C" int pd_timing_enable(int32_t enable)
{
    clear_timing();
    g_timing = enable != 0;
    return PD_OK;
}

extern "C" int pd_timing_read(int32_t max_rows, int32_t *kclass, int32_t *level, int64_t *launches,
                              double *total_ms, int32_t *rows)
{
    if (!rows || max_rows < 0) return PD_ERR_ARG;
    std::map<std::pair<int, int>, std::pair<int64_t, double>> agg;
    for (auto &t : g_launches) {
        if (hipEventSynchronize(t.b) != hipSuccess) return PD_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess) return PD_ERR_HIP;
        auto &e = agg[{t.kclass, t.level}];
        e.first += 1;
        e.second += ms;
    }
    int r = 0;
    for (auto &kv : agg) {
        if (r < max_rows) {
            if (kclass) kclass[r] = kv.first.first;
            if (level) level[r] = kv.first.second;
            if (launches) launches[r] = kv.second.first;
            if (total_ms) total_ms[r] = kv.second.second;
        }
        ++r;
    }
    *rows = r;
    return PD_OK;
}

extern "C" size_t pd_workspace_size(const pd_shape *shape, int32_t dtype)
{
    if (check_shape(shape) != PD_OK || check_dtype(dtype) != PD_OK) return 0;
    return layout(shape, dtype == PD_F64 ? 8 : 4).total;
}

namespace {

int solve_checked(const pd_shape *shape, int32_t dtype, const pd_operator *op, const pd_wavelet *wav,
                  const pd_weights *w, const pd_params *prm, const void *f0, void *z_cur, void *z_prev,
                  int32_t init_from_f0, void *f_out, double *stats, void *workspace, size_t ws_bytes,
                  void *stream, bool eager)
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
                                 ws_bytes, st, eager);
    return solve_impl<double>(shape, op, wav, w, prm, (const double *)f0, (double *)z_cur,
                              (double *)z_prev, init_from_f0, (double *)f_out, stats, workspace,
                              ws_bytes, st, eager);
}

// ------------------------------------------------------ allocation-free --
// pd_solve_noalloc's scratch: a fixed device array in this library's code
// object (one copy per GPU, alive until the process ends).  Host code never
// passes `scratch` itself to a kernel (its host-side name is not a device
// address): the device address is taken once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t NOALLOC_BYTES = (size_t)PD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

int scratch_address(void **out)
{
    int dev = 0;
    PD_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return PD_ERR_HIP;
        }
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return PD_OK;
}

}  // namespace

extern "C" int pd_solve(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                        const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                        const void *f0, void *z_cur, void *z_prev, int32_t init_from_f0,
                        void *f_out, double *stats, void *workspace, size_t ws_bytes,
                        void *stream)
{
    return solve_checked(shape, dtype, op, wav, w, prm, f0, z_cur, z_prev, init_from_f0, f_out, stats,
                         workspace, ws_bytes, stream, false);
}

extern "C" int pd_solve_noalloc(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                                const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                                const void *f0, void *z_cur, void *z_prev, int32_t init_from_f0,
                                void *f_out, double *stats, void *stream)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype))) return rc;
    if (layout(shape, dtype == PD_F64 ? 8 : 4).total > NOALLOC_BYTES) return PD_ERR_WORKSPACE;
    void *ws = nullptr;
    if ((rc = scratch_address(&ws)) != PD_OK) return rc;
    return solve_checked(shape, dtype, op, wav, w, prm, f0, z_cur, z_prev, init_from_f0, f_out, stats, ws,
                         NOALLOC_BYTES, stream, true);
}

extern "C" int pd_tune(const pd_shape *shape, int32_t dtype, const pd_operator *op, void *workspace,
                       size_t ws_bytes, int32_t *chosen, void *stream)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype)) || (rc = check_op(op, shape))) return rc;
    if (!workspace) return PD_ERR_ARG;
    const size_t es = dtype == PD_F64 ? 8 : 4;
    const Layout lay = layout(shape, es);
    if (ws_bytes < lay.total) return PD_ERR_WORKSPACE;
    const int pin = chosen ? *chosen : 0;
    if (chosen) *chosen = 0;
    if (op->kind != PD_OP_ROWBLUR) return PD_OK;  // nothing tunable for the other operators
    for (int v : BLUR_VARIANTS)
        if (pin == v) {  // a variant named by the caller: recorded without timing
            set_blur_variant(shape->n1, shape->n2, shape->channels, op->radius, (int)es, v);
            *chosen = v;
            return PD_OK;
        }
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    const int n1 = shape->n1, n2 = shape->n2, C = shape->channels, R = op->radius;
    const int64_t NC = (int64_t)n1 * n2 * C;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Events {
        hipEvent_t &a, &b;
        ~Events()
        {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    PD_TRY_HIP(hipEventCreate(&e0));
    PD_TRY_HIP(hipEventCreate(&e1));
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        // the blur of a zero plane into the solver's s plane (no statistics): timing only
        T *x = (T *)(ws + lay.x), *sp = (T *)(ws + lay.s);
        PD_TRY_HIP(launch_fill<T>(x, T(0), NC, st));
        BlurArgs<T> a{};
        a.x = x;
        a.f0 = nullptr;
        a.s = sp;
        a.taps = (const T *)op->taps;
        a.n1 = n1;
        a.n2 = n2;
        a.C = C;
        a.R = R;
        a.plane = (int64_t)n1 * n2;
        a.slots = nullptr;
        a.racc = nullptr;
        a.rscale = T(0);
        a.r = (T *)(ws + lay.r);
        a.tabs = (T *)(ws + lay.btab);
        a.rows = 0;
        PD_TRY_HIP(launch_blur_tables<T>((const T *)op->taps, n2, R, (T *)(ws + lay.btab), st));
        float best_ms = 0.0f;
        int best = BLUR_VARIANTS[0];
        for (int v : BLUR_VARIANTS) {
            set_blur_variant(n1, n2, C, R, (int)es, v);
            for (int k = 0; k < 3; ++k) PD_TRY_HIP(launch_blur<T>(a, false, st));
            PD_TRY_HIP(hipEventRecord(e0, st));
            for (int k = 0; k < 10; ++k) PD_TRY_HIP(launch_blur<T>(a, false, st));
            PD_TRY_HIP(hipEventRecord(e1, st));
            PD_TRY_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            PD_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (v == BLUR_VARIANTS[0] || ms < best_ms) {
                best_ms = ms;
                best = v;
            }
        }
        set_blur_variant(n1, n2, C, R, (int)es, best);
        if (chosen) *chosen = best;
        return PD_OK;
    };
    return dtype == PD_F32 ? run(float(0)) : run(double(0));
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
        if (ws_bytes < layout(shape, sizeof(T)).total) return PD_ERR_WORKSPACE;
        Ctx<T> c = make_ctx<T>(shape, wav, workspace, st, 0);
        if (inverse) return synth_chain<T>(c, (const T *)in, (const T *)in, T(0), (T *)out);
        return analysis_plain<T>(c, (const T *)in, (T *)out);
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
        if (op->kind == PD_OP_PC) {
            PcArgs<T> p{(const T *)in, nullptr, (T *)out, (const T *)op->taps, (const T *)op->mult, shape->n1,
                        shape->n2, shape->channels, op->radius, op->terms, (int64_t)shape->n1 * shape->n2, nullptr};
            PD_TRY_HIP(launch_pc_single<T>(p, transpose, st));
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
        a.slots = nullptr;
        a.racc = nullptr;
        a.rscale = T(0);
        PD_TRY_HIP(launch_blur_single<T>(a, transpose, st));
        return PD_OK;
    };
    return dtype == PD_F32 ? run(float(0)) : run(double(0));
}

// --------------------------------------------------------------- backward --
// Reverse mode of pd_solve (init = Psi^* f0) with segment checkpointing:
// forward pass storing (z(sC), z(sC-1)) at the start of every segment of C
// iterations; then, last segment first, the segment's z(i) are recomputed from
// its checkpoint by the same launch sequence as the forward solve (bitwise the
// same iterates) and the adjoint recursion is run backwards through it:
//   zbar(K) = Psi^* fbar
//   vbar = zbar 1{z(i) != 0};  wbar -= tau zbar sign z(i)
//   ybar = vbar - tau Psi^* H^T H Psi vbar;  f0bar += tau H Psi vbar
//   zbar(i-1) = zbarm + (1+b) ybar,  zbarm = -b ybar,  b = (i-2)/(i+1)
//   f0bar += Psi (ybar(1) + zbarm)                       (adjoint of the init)
namespace {

struct BwdLayout {
    Layout fwd;
    int nseg;
    size_t zc, zp, ck, seg, zbar, zbarm, vbar, gbar, total;
};

BwdLayout bwd_layout(const pd_shape *sh, size_t es, int iters, int C)
{
    BwdLayout b;
    b.fwd = layout(sh, es);
    b.nseg = iters > 0 ? (iters + C - 1) / C : 0;
    const size_t plane = align_up(es * (size_t)sh->n1 * sh->n2 * sh->channels);
    size_t off = b.fwd.total;
    b.zc = off;
    off += plane;
    b.zp = off;
    off += plane;
    b.ck = off;
    off += plane * 2 * (size_t)b.nseg;
    b.seg = off;
    off += plane * (size_t)(iters > 0 ? std::min(C, iters) : 0);
    b.zbar = off;
    off += plane;
    b.zbarm = off;
    off += plane;
    b.vbar = off;
    off += plane;
    b.gbar = off;
    off += plane;
    b.total = off;
    return b;
}

// The forward recursion from z(0) = Psi^* f0 with (z(i), z(i-1)) stored at
// the start of every segment of C iterations in the checkpoint area of a
// backward workspace.  With f_out, every segment is run and f = Psi z(K)
// written; without, the last segment is left to the reverse sweep (which
// recomputes it first anyway).
template <typename T>
int forward_checkpoints(const Ctx<T> &c, const BwdLayout &L, const pd_operator *op, const pd_weights *w, T tau,
                        int K, int C, const T *f0, T *f_out)
{
    char *ws = c.ws;
    const hipStream_t st = c.st;
    const int64_t NC = c.N() * c.sh->channels;
    const size_t plane = align_up(sizeof(T) * (size_t)NC);
    T *zA = (T *)(ws + L.zc), *zB = (T *)(ws + L.zp);
    auto ck = [&](int sidx, int k) { return (T *)(ws + L.ck + plane * (2 * (size_t)sidx + k)); };
    int rc;
    if ((rc = analysis_plain<T>(c, f0, zA)) != PD_OK) return rc;
    PD_TRY_HIP(launch_copy<T>(zA, zB, NC, st));
    T *zc = zA, *zp = zB;
    for (int sidx = 0; sidx < L.nseg; ++sidx) {
        PD_TRY_HIP(launch_copy<T>(zc, ck(sidx, 0), NC, st));
        PD_TRY_HIP(launch_copy<T>(zp, ck(sidx, 1), NC, st));
        const int i0 = sidx * C + 1, cnt = std::min(C, K - sidx * C);
        if (sidx == L.nseg - 1 && !f_out) break;
        if ((rc = iterate<T>(c, op, w, tau, f0, zc, zp, i0, cnt, nullptr, nullptr)) != PD_OK) return rc;
    }
    if (f_out) return synth_chain<T>(c, zc, zc, T(0), f_out);  // zc = z(K)
    return PD_OK;
}

template <typename T>
int forward_ck_impl(const pd_shape *sh, const pd_operator *op, const pd_wavelet *wav, const pd_weights *w,
                    const pd_params *prm, const T *f0, T *f_out, int C, void *workspace, size_t ws_bytes,
                    hipStream_t st)
{
    const BwdLayout L = bwd_layout(sh, sizeof(T), prm->iters, C);
    if (ws_bytes < L.total) return PD_ERR_WORKSPACE;
    Ctx<T> c = make_ctx<T>(sh, wav, workspace, st, 0);
    int rc;
    if ((rc = prep_blur<T>(c, op)) != PD_OK) return rc;
    return forward_checkpoints<T>(c, L, op, w, (T)prm->tau, prm->iters, C, f0, f_out);
}

template <typename T>
int backward_impl(const pd_shape *sh, const pd_operator *op, const pd_wavelet *wav, const pd_weights *w,
                  const pd_params *prm, const T *f0, const T *gf, T *gf0, T *gw, int C, void *workspace,
                  size_t ws_bytes, hipStream_t st, bool have_checkpoints)
{
    const int K = prm->iters;
    BwdLayout L = bwd_layout(sh, sizeof(T), K, C);
    if (ws_bytes < L.total) return PD_ERR_WORKSPACE;
    Ctx<T> c = make_ctx<T>(sh, wav, workspace, st, 0);
    char *ws = (char *)workspace;
    const int64_t NC = c.N() * sh->channels;
    const size_t plane = align_up(sizeof(T) * (size_t)NC);
    T *zA = (T *)(ws + L.zc), *zB = (T *)(ws + L.zp);
    T *zbar = (T *)(ws + L.zbar), *zbarm = (T *)(ws + L.zbarm);
    T *vbar = (T *)(ws + L.vbar), *gbar = (T *)(ws + L.gbar);
    auto ck = [&](int sidx, int k) { return (T *)(ws + L.ck + plane * (2 * (size_t)sidx + k)); };
    T *seg = (T *)(ws + L.seg);
    const T tau = (T)prm->tau;
    int rc;
    if ((rc = prep_blur<T>(c, op)) != PD_OK) return rc;

    // forward with checkpoints (unless pd_solve_checkpointed left them in this workspace)
    if (!have_checkpoints && (rc = forward_checkpoints<T>(c, L, op, w, tau, K, C, f0, nullptr)) != PD_OK)
        return rc;
    // seeds
    if ((rc = analysis_plain<T>(c, gf, zbar)) != PD_OK) return rc;  // zbar(K) = Psi^* fbar
    PD_TRY_HIP(launch_fill<T>(zbarm, T(0), NC, st));
    if (gf0) PD_TRY_HIP(launch_fill<T>(gf0, T(0), NC, st));
    if (gw) PD_TRY_HIP(launch_fill<T>(gw, T(0), NC, st));

    // One segment: recompute its iterates from (zc, zp), then run the adjoint
    // back through them.  With di set, i comes from device memory (*it_dev is
    // the segment's first iteration) so that a captured graph of a full
    // segment replays for every full segment.
    auto segment = [&](const Ctx<T> &cs, T *zc, T *zp, int i0, int cnt, bool dev) -> int {
        const hipStream_t s = cs.st;
        if ((rc = iterate_seg<T>(cs, op, w, tau, f0, zc, zp, i0, cnt, seg, dev ? cs.it_dev() : nullptr)) != PD_OK)
            return rc;
        // The mask of iteration j-1 runs in the same launch as the combine of j.
        // With a coarse block, iterations j > 0 end with one coarse launch: the
        // analysis of gbar on the block, combine and mask there, and the
        // synthesis of the next vbar (the element-wise launch skips the block),
        // so the next iteration synthesises the fine levels only.
        const bool fco = g_synth2 && cs.lc <= cs.sh->levels;
        const int cm1 = cs.sh->n1 >> (cs.lc - 1), cm2 = cs.sh->n2 >> (cs.lc - 1);
        if (cnt > 0) PD_TRY_HIP(launch_rev_mask<T>(zbar, seg + (int64_t)(cnt - 1) * NC, vbar, gw, tau, NC, s));
        for (int j = cnt - 1; j >= 0; --j) {
            const int i = i0 + j;
            if (fco && j < cnt - 1) {
                if ((rc = synth_fine<T>(cs, vbar, vbar, T(0), cs.x())) != PD_OK) return rc;      // Psi vbar
            } else if ((rc = synth_chain<T>(cs, vbar, vbar, T(0), cs.x())) != PD_OK) {
                return rc;
            }
            if ((rc = blur_step<T>(cs, op, cs.x(), nullptr, cs.s(), nullptr, gf0, tau)) != PD_OK) return rc;
            const T b = (T)beta_y(i);  // b_{i-1}
            const DevIter di{dev ? cs.it_dev() : nullptr, j};
            if (j > 0 && fco) {
                // Psi^* H^T H Psi vbar: the fine levels, then the block in the coarse launch
                ProxArgs<T> pl = prox_args<T>(cs, nullptr, nullptr, gbar, T(0), T(0), nullptr, nullptr);
                if ((rc = analysis_fine<T>(cs, cs.s(), MODE_PLAIN, pl)) != PD_OK) return rc;
                ProxArgs<T> pr = prox_args<T>(cs, vbar, seg + (int64_t)(j - 1) * NC, gbar, T(0), tau, nullptr, nullptr);
                CoarseArgs<T> rv;
                rv.rv_vbar = vbar;
                rv.rv_zbar = zbar;
                rv.rv_zbarm = zbarm;
                rv.rv_wbar = gw;
                rv.rv_b = b;
                rv.rv_first = i == 1 ? 1 : 0;
                rv.rv_di = di;
                if ((rc = coarse_step<T>(cs, COARSE_ANA | COARSE_REVCM | COARSE_SYN, cs.s(), cs.x(), pr, T(0), &rv)) !=
                    PD_OK)
                    return rc;
                PD_TRY_HIP(launch_rev_combine_mask<T>(vbar, gbar, zbar, zbarm, seg + (int64_t)(j - 1) * NC, gw, tau, b,
                                                      i == 1 ? 1 : 0, NC, di, cm1, cm2, cs.sh->n1, cs.N(), s));
                continue;
            }
            if ((rc = analysis_plain<T>(cs, cs.s(), gbar)) != PD_OK) return rc;                   // Psi^* H^T H Psi vbar
            if (j > 0)
                PD_TRY_HIP(launch_rev_combine_mask<T>(vbar, gbar, zbar, zbarm, seg + (int64_t)(j - 1) * NC, gw, tau, b,
                                                      i == 1 ? 1 : 0, NC, di, 0, 0, cs.sh->n1, cs.N(), s));
            else
                PD_TRY_HIP(launch_rev_combine<T>(vbar, gbar, zbar, zbarm, tau, b, i == 1 ? 1 : 0, NC, di, s));
        }
        return PD_OK;
    };
    // full segments other than the last: one captured graph, replayed from
    // the working planes zA, zB (the checkpoint is copied there first)
    hipGraphExec_t seg_graph = nullptr;
    const int full = (L.nseg > 1 && g_graphs && !g_timing) ? L.nseg - 1 : 0;
    {
        std::lock_guard<std::mutex> lock(g_graph_mu);
        sweep_retired();
    }
    if (full >= 2) {
        int dev = 0;
        hipStream_t cap = nullptr;
        if (hipGetDevice(&dev) == hipSuccess) {
            std::lock_guard<std::mutex> lock(g_graph_mu);
            cap = capture_stream(dev);
        }
        if (cap) {
            Ctx<T> cs = c;
            cs.st = cap;
            if (hipStreamBeginCapture(cs.st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                const int crc = segment(cs, zA, zB, 1, C, true);
                hipGraph_t g = nullptr;
                const hipError_t e = hipStreamEndCapture(cs.st, &g);
                if (crc == PD_OK && e == hipSuccess && g &&
                    hipGraphInstantiate(&seg_graph, g, nullptr, nullptr, 0) != hipSuccess)
                    seg_graph = nullptr;
                if (g) (void)hipGraphDestroy(g);
            }
            (void)hipGetLastError();
        }
    }
    // every segment recomputes from a copy of its checkpoint in the working
    // planes (the recursion runs in place), so the checkpoints stay intact for
    // another reverse sweep (pd_backward_checkpointed)
    for (int sidx = L.nseg - 1; sidx >= 0; --sidx) {
        const int i0 = sidx * C + 1, cnt = std::min(C, K - sidx * C);
        PD_TRY_HIP(launch_copy<T>(ck(sidx, 0), zA, NC, st));
        PD_TRY_HIP(launch_copy<T>(ck(sidx, 1), zB, NC, st));
        if (seg_graph && sidx < L.nseg - 1) {
            PD_TRY_HIP(launch_set_int(c.it_dev(), i0, st));
            PD_TRY_HIP(hipGraphLaunch(seg_graph, st));
            continue;
        }
        if ((rc = segment(c, zA, zB, i0, cnt, false)) != PD_OK) return rc;
    }
    if (seg_graph) {  // retired: destroyed once its last launch has run
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(ev, st) == hipSuccess) {
            std::lock_guard<std::mutex> lock(g_graph_mu);
            g_graph_retired.push_back(CachedGraph{{}, seg_graph, ev});
        } else {
            PD_TRY_HIP(hipStreamSynchronize(st));
            (void)hipGraphExecDestroy(seg_graph);
            if (ev) (void)hipEventDestroy(ev);
        }
    }
    // f0bar += Psi initbar (initbar = zbar after the i = 1 step, or Psi^* fbar when K = 0)
    if (gf0) {
        if ((rc = synth_chain<T>(c, zbar, zbar, T(0), c.x())) != PD_OK) return rc;
        PD_TRY_HIP(launch_add<T>(c.x(), gf0, NC, st));
    }
    return PD_OK;
}

}  // namespace

extern "C" size_t pd_backward_workspace_size(const pd_shape *shape, int32_t dtype, int32_t iters,
                                             int32_t checkpoint_every)
{
    if (check_shape(shape) != PD_OK || check_dtype(dtype) != PD_OK || iters < 0 || checkpoint_every < 1) return 0;
    return bwd_layout(shape, dtype == PD_F64 ? 8 : 4, iters, checkpoint_every).total;
}

namespace {

int check_backward(const pd_shape *shape, int32_t dtype, const pd_operator *op, const pd_wavelet *wav,
                   const pd_weights *w, const pd_params *prm, const void *f0, int32_t checkpoint_every,
                   void *workspace)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype)) || (rc = check_op(op, shape)) ||
        (rc = check_wavelet(wav)) || (rc = check_weights(w, shape)) || (rc = check_params(prm)))
        return rc;
    if (!f0 || !workspace || checkpoint_every < 1) return PD_ERR_ARG;
    if (w->joint || prm->iter_offset != 0 || op->kind == PD_OP_PC) return PD_ERR_UNSUPPORTED;
    return PD_OK;
}

int backward_checked(const pd_shape *shape, int32_t dtype, const pd_operator *op, const pd_wavelet *wav,
                     const pd_weights *w, const pd_params *prm, const void *f0, const void *grad_f, void *grad_f0,
                     void *grad_w, int32_t checkpoint_every, void *workspace, size_t ws_bytes, void *stream,
                     bool have_checkpoints)
{
    int rc;
    if ((rc = check_backward(shape, dtype, op, wav, w, prm, f0, checkpoint_every, workspace))) return rc;
    if (!grad_f) return PD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PD_F32)
        return backward_impl<float>(shape, op, wav, w, prm, (const float *)f0, (const float *)grad_f,
                                    (float *)grad_f0, (float *)grad_w, checkpoint_every, workspace, ws_bytes, st,
                                    have_checkpoints);
    return backward_impl<double>(shape, op, wav, w, prm, (const double *)f0, (const double *)grad_f,
                                 (double *)grad_f0, (double *)grad_w, checkpoint_every, workspace, ws_bytes, st,
                                 have_checkpoints);
}

}  // namespace

extern "C" int pd_backward(const pd_shape *shape, int32_t dtype, const pd_operator *op, const pd_wavelet *wav,
                           const pd_weights *w, const pd_params *prm, const void *f0, const void *grad_f,
                           void *grad_f0, void *grad_w, int32_t checkpoint_every, void *workspace,
                           size_t ws_bytes, void *stream)
{
    return backward_checked(shape, dtype, op, wav, w, prm, f0, grad_f, grad_f0, grad_w, checkpoint_every, workspace,
                            ws_bytes, stream, false);
}

extern "C" int pd_solve_checkpointed(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                                     const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                                     const void *f0, void *f_out, int32_t checkpoint_every, void *workspace,
                                     size_t ws_bytes, void *stream)
{
    int rc;
    if ((rc = check_backward(shape, dtype, op, wav, w, prm, f0, checkpoint_every, workspace))) return rc;
    if (!f_out || f_out == f0) return PD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PD_F32)
        return forward_ck_impl<float>(shape, op, wav, w, prm, (const float *)f0, (float *)f_out, checkpoint_every,
                                      workspace, ws_bytes, st);
    return forward_ck_impl<double>(shape, op, wav, w, prm, (const double *)f0, (double *)f_out, checkpoint_every,
                                   workspace, ws_bytes, st);
}

extern "C" int pd_backward_checkpointed(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                                        const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                                        const void *f0, const void *grad_f, void *grad_f0, void *grad_w,
                                        int32_t checkpoint_every, void *workspace, size_t ws_bytes, void *stream)
{
    return backward_checked(shape, dtype, op, wav, w, prm, f0, grad_f, grad_f0, grad_w, checkpoint_every, workspace,
                            ws_bytes, stream, true);
}

// ------------------------------------------------------------------ ADMM-PC --
// ADMM on eq. 4.1 with a product-convolution operator H = U V (Appendix A.2):
// g = (U^T U + beta1 D)^-1 (U^T f0 - xi + beta1 D V f) by the Woodbury
// identity in the Fourier basis, z = Prox(Psi^* f - zeta / beta2), f by its
// diagonal normal equations, then the multiplier updates; beta1 = beta2 =
// beta, gamma_k = max|u_k^| normalised to sum 1, start f = f0, z = Psi^* f0,
// xi = zeta = 0.  Channels are solved one after the other (same operator).
namespace {

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

struct AdmmLayout {
    size_t zeta, g, xi, utf0, den, mh, tz, tfz, tfs, uh, cb, th, tw1, tw2, gam, mx, total;
};

AdmmLayout admm_layout(const pd_shape *sh, size_t es, int m)
{
    pd_shape s1 = *sh;
    s1.channels = 1;
    const size_t N = (size_t)sh->n1 * sh->n2;
    AdmmLayout l;
    size_t off = align_up(layout(&s1, es).total);
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.zeta = take(N * es);
    l.g = take((size_t)m * N * es);
    l.xi = take((size_t)m * N * es);
    l.utf0 = take((size_t)m * N * es);
    l.den = take(N * es);
    l.mh = take(N * es);
    l.tz = take(N * es);
    l.tfz = take(N * es);
    l.tfs = take(N * es);
    l.uh = take((size_t)m * N * 2 * es);
    l.cb = take((size_t)m * N * 2 * es);
    l.th = take(N * 2 * es);
    l.tw1 = take((size_t)sh->n1 * es);   // n1/2 complex
    l.tw2 = take((size_t)sh->n2 * es);
    l.gam = take((size_t)m * es);
    l.mx = take((size_t)m * es);
    l.total = off;
    return l;
}

// A second, library-owned stream per device (default priority), for work that runs beside the
// caller's stream inside one call.  Each call orders its work with events of its own (concurrent
// calls never record each other's events) and joins the side stream back into the caller's stream
// on every return path.
std::mutex g_side_mu;

hipStream_t side_stream()
{
    static std::map<int, hipStream_t> side;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_side_mu);
    auto it = side.find(dev);
    if (it == side.end()) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
        it = side.emplace(dev, s).first;
    }
    return it->second;
}

struct SideCall {
    hipStream_t s = nullptr, st = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
    bool open(hipStream_t caller)
    {
        st = caller;
        s = side_stream();
        return s && hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess;
    }
    ~SideCall()
    {
        if (s && done && hipEventRecord(done, s) == hipSuccess) (void)hipStreamWaitEvent(st, done, 0);
        if (ready) (void)hipEventDestroy(ready);
        if (done) (void)hipEventDestroy(done);
    }
};

template <typename T>
int admm_impl(const pd_shape *sh, const pd_operator *op, const pd_wavelet *wav, const pd_weights *w, double beta,
              int iters, const T *f0, T *f_out, T *z_out, double *stats, void *workspace, size_t ws_bytes,
              hipStream_t st)
{
    const int n1 = sh->n1, n2 = sh->n2, m = op->terms;
    const int64_t N = (int64_t)n1 * n2;
    const AdmmLayout L = admm_layout(sh, sizeof(T), m);
    if (ws_bytes < L.total) return PD_ERR_WORKSPACE;
    char *ws = (char *)workspace;
    pd_shape s1 = *sh;
    s1.channels = 1;
    Ctx<T> c = make_ctx<T>(&s1, wav, workspace, st, 0);
    if (c.ts.nt > 0 && !c.tail) return PD_ERR_HIP;
    SideCall side;
    if (!side.open(st)) return PD_ERR_HIP;
    Ctx<T> c2 = c;  // the same transforms and scratch, launched on the side stream
    c2.st = side.s;
    AdmmArgs<T> a{};
    a.n1 = n1;
    a.n2 = n2;
    a.m = m;
    a.levels = sh->levels;
    a.N = N;
    a.beta1 = a.beta2 = (T)beta;
    a.gam = (const T *)(ws + L.gam);
    a.v = (const T *)op->mult;
    a.uh = (const Cx<T> *)(ws + L.uh);
    a.mh = (const T *)(ws + L.mh);
    a.den = (const T *)(ws + L.den);
    a.utf0 = (const T *)(ws + L.utf0);
    a.g = (T *)(ws + L.g);
    a.xi = (T *)(ws + L.xi);
    a.zeta = (T *)(ws + L.zeta);
    a.tz = (T *)(ws + L.tz);
    a.cb = (Cx<T> *)(ws + L.cb);
    a.tf = (T *)(ws + L.tfz);
    a.tfs = (const T *)(ws + L.tfs);
    a.wmap = (const T *)w->coeff_w;
    for (int k = 0; k <= PD_MAXL; ++k) a.wlev[k] = (w->level_w && k <= sh->levels) ? (T)w->level_w[k] : T(0);
    T *tfz = (T *)(ws + L.tfz), *tfs = (T *)(ws + L.tfs);
    Cx<T> *th = (Cx<T> *)(ws + L.th);
    Cx<T> *tw1 = (Cx<T> *)(ws + L.tw1), *tw2 = (Cx<T> *)(ws + L.tw2);
    Cx<T> *uh = (Cx<T> *)(ws + L.uh);

    // twiddles, kernel spectra, gamma_k = ||U_k|| normalised to sum 1, diagonal factors
    PD_TRY_HIP(launch_admm_twiddle<T>(tw1, n1, st));
    PD_TRY_HIP(launch_admm_twiddle<T>(tw2, n2, st));
    PD_TRY_HIP(launch_admm_padk<T>((const T *)op->taps, op->radius, m, n1, n2, uh, st));
    PD_TRY_HIP(launch_fft2<T>(uh, n1, n2, m, tw1, tw2, 0, st));
    PD_TRY_HIP(launch_admm_absmax<T>(uh, m, N, (T *)(ws + L.mx), st));
    PD_TRY_HIP(launch_admm_gamma<T>((const T *)(ws + L.mx), m, (T *)(ws + L.gam), st));
    PD_TRY_HIP(launch_admm_diag<T>(a, st));

    if (stats && iters > 0) PD_TRY_HIP(launch_fill<double>(stats, 0.0, (int64_t)iters * 3, st));
    for (int ch = 0; ch < sh->channels; ++ch) {
        const T *f0c = f0 + ch * N;
        a.f = f_out + ch * N;
        a.z = z_out + ch * N;
        // U_k^T f0 through the spectra (all k at once)
        PD_TRY_HIP(launch_admm_real<T>(f0c, th, N, st));
        PD_TRY_HIP(launch_fft2<T>(th, n1, n2, 1, tw1, tw2, 0, st));
        PD_TRY_HIP(launch_admm_conjmul<T>(uh, th, a.cb, m, N, st));
        PD_TRY_HIP(launch_fft2<T>(a.cb, n1, n2, m, tw1, tw2, 1, st));
        PD_TRY_HIP(launch_admm_takere<T>(a.cb, (T *)a.utf0, (int64_t)m * N, st));
        // start: f = f0, z = Psi^* f, xi = zeta = 0; first a_k and z
        PD_TRY_HIP(launch_copy<T>(f0c, a.f, N, st));
        int rc;
        if ((rc = analysis_plain<T>(c, a.f, a.tz)) != PD_OK) return rc;
        PD_TRY_HIP(launch_fill<T>(a.zeta, T(0), N, st));
        PD_TRY_HIP(launch_fill<T>(a.xi, T(0), (int64_t)m * N, st));
        if (iters == 0) {
            PD_TRY_HIP(launch_copy<T>(a.tz, a.z, N, st));
            continue;
        }
        if (stats) PD_TRY_HIP(launch_fill<double>(c.ring(), 0.0, (int64_t)PD_RING * 3 * PD_NSLOT, st));
        a.slots = stats ? c.slots(0) : nullptr;
        PD_TRY_HIP(launch_admm_a<T>(a, st));
        PD_TRY_HIP(launch_admm_z<T>(a, st));
        int b0 = 0;
        // timed launches: FFT passes keyed 0/1 (forward rows/columns), 2/3 (inverse); element-wise
        // steps 1 (spectral), 2 (f and multipliers), 3 (zeta and z)
        auto fft = [&](int inverse) -> int {
            for (int cols = 0; cols < 2; ++cols)
                PD_TRY_HIP(timed(PD_K_FFT, 2 * inverse + cols, st, [&] {
                    return launch_fft_pass<T>(a.cb, n1, n2, m, cols ? tw2 : tw1, inverse, cols, st);
                }));
            return PD_OK;
        };
        // Two streams.  The caller's stream runs the g-step (FFTs and the spectral product) and
        // the f-step; the side stream runs, after each f-step, the analysis of f, the zeta / z
        // step and the synthesis of the next beta2 z + zeta.  Neither stream touches the other's
        // buffers between the joins: the g-step reads and writes the complex planes, the side
        // chain f, z, zeta, Psi^* f, the synthesis buffers and the transforms' scratch pyramid;
        // the f-step (after a join) reads the synthesis and writes f and the next a_k.
        PD_TRY_HIP(hipEventRecord(side.ready, st));
        PD_TRY_HIP(hipStreamWaitEvent(side.s, side.ready, 0));
        if ((rc = synth_chain<T>(c2, tfz, tfz, T(0), tfs)) != PD_OK) return rc;
        PD_TRY_HIP(hipEventRecord(side.done, side.s));
        for (int it = 0; it < iters; ++it) {
            const int next = it + 1 < iters;
            a.slots = stats ? c.slots(it) : nullptr;
            a.slots_next = (stats && next) ? c.slots(it + 1) : nullptr;
            // g: Woodbury with the Fourier-diagonal middle matrix (a_k already in g and cb)
            if ((rc = fft(0)) != PD_OK) return rc;
            PD_TRY_HIP(timed(PD_K_ADMM, 1, st, [&] { return launch_admm_accq<T>(a, st); }));
            if ((rc = fft(1)) != PD_OK) return rc;
            // f (the z of this iteration was formed with the previous multiplier step), multipliers
            PD_TRY_HIP(hipStreamWaitEvent(st, side.done, 0));
            PD_TRY_HIP(timed(PD_K_ADMM, 2, st, [&] { return launch_admm_f<T>(a, next, st); }));
            PD_TRY_HIP(hipEventRecord(side.ready, st));
            PD_TRY_HIP(hipStreamWaitEvent(side.s, side.ready, 0));
            if ((rc = analysis_plain<T>(c2, a.f, a.tz)) != PD_OK) return rc;
            PD_TRY_HIP(timed(PD_K_ADMM, 3, side.s, [&] { return launch_admm_zeta<T>(a, next, side.s); }));
            // batches of at most PD_RING - 1 entries, so that the entry of iteration it + 1 (whose
            // penalty term is already in the ring) is never finalised with an older one
            if (stats && (it + 1 - b0 == PD_RING - 1 || it == iters - 1)) {
                PD_TRY_HIP(launch_stats_finalize(c.ring(), stats, b0, it + 1 - b0, side.s));
                b0 = it + 1;
            }
            if (next && (rc = synth_chain<T>(c2, tfz, tfz, T(0), tfs)) != PD_OK) return rc;
            PD_TRY_HIP(hipEventRecord(side.done, side.s));
        }
        PD_TRY_HIP(hipStreamWaitEvent(st, side.done, 0));  // join before the next channel / return
    }
    return PD_OK;
}

}  // namespace

extern "C" size_t pd_admm_workspace_size(const pd_shape *shape, int32_t dtype, int32_t terms)
{
    if (check_shape(shape) != PD_OK || check_dtype(dtype) != PD_OK || terms < 1 || terms > PD_MAX_PC) return 0;
    return admm_layout(shape, dtype == PD_F64 ? 8 : 4, terms).total;
}

extern "C" int pd_admm_solve(const pd_shape *shape, int32_t dtype, const pd_operator *op, const pd_wavelet *wav,
                             const pd_weights *w, double beta, int32_t iters, const void *f0, void *f_out,
                             void *z_out, double *stats, void *workspace, size_t ws_bytes, void *stream)
{
    int rc;
    if ((rc = check_shape(shape)) || (rc = check_dtype(dtype)) || (rc = check_op(op, shape)) ||
        (rc = check_wavelet(wav)) || (rc = check_weights(w, shape)))
        return rc;
    if (op->kind != PD_OP_PC || w->joint) return PD_ERR_UNSUPPORTED;
    const int nmax = dtype == PD_F64 ? 2048 : 4096;  // one FFT line and its ping-pong copy within 64 KiB of LDS
    if (!pow2_in(shape->n1, 2, nmax) || !pow2_in(shape->n2, 2, nmax)) return PD_ERR_UNSUPPORTED;
    if (!std::isfinite(beta) || beta <= 0.0) return PD_ERR_TAU;
    if (iters < 0 || !f0 || !f_out || !z_out || !workspace) return PD_ERR_ARG;
    if (f0 == f_out || f0 == z_out || f_out == z_out) return PD_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (dtype == PD_F32)
        return admm_impl<float>(shape, op, wav, w, beta, iters, (const float *)f0, (float *)f_out, (float *)z_out,
                                stats, workspace, ws_bytes, st);
    return admm_impl<double>(shape, op, wav, w, beta, iters, (const double *)f0, (double *)f_out, (double *)z_out,
                             stats, workspace, ws_bytes, st);
}

extern "C" size_t pd_fft2_workspace_size(int32_t n1, int32_t n2, int32_t dtype)
{
    if (check_dtype(dtype) != PD_OK) return 0;
    const int nmax = dtype == PD_F64 ? 2048 : 4096;
    if (!pow2_in(n1, 2, nmax) || !pow2_in(n2, 2, nmax)) return 0;
    const size_t es = dtype == PD_F64 ? 8 : 4;
    return align_up((size_t)n1 * es) + align_up((size_t)n2 * es);
}

extern "C" int pd_fft2(int32_t n1, int32_t n2, int32_t batch, int32_t dtype, int32_t inverse, void *data,
                       void *workspace, size_t ws_bytes, void *stream)
{
    int rc;
    if ((rc = check_dtype(dtype))) return rc;
    const int nmax = dtype == PD_F64 ? 2048 : 4096;
    if (!pow2_in(n1, 2, nmax) || !pow2_in(n2, 2, nmax)) return PD_ERR_UNSUPPORTED;
    if (batch < 0 || (batch > 0 && (!data || !workspace))) return PD_ERR_ARG;
    if (batch == 0) return PD_OK;
    if (ws_bytes < pd_fft2_workspace_size(n1, n2, dtype)) return PD_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const size_t es = dtype == PD_F64 ? 8 : 4, o2 = align_up((size_t)n1 * es);
    char *ws = (char *)workspace;
    if (dtype == PD_F32) {
        Cx<float> *t1 = (Cx<float> *)ws, *t2 = (Cx<float> *)(ws + o2);
        PD_TRY_HIP(launch_admm_twiddle<float>(t1, n1, st));
        PD_TRY_HIP(launch_admm_twiddle<float>(t2, n2, st));
        PD_TRY_HIP(launch_fft2<float>((Cx<float> *)data, n1, n2, batch, t1, t2, inverse != 0, st));
    } else {
        Cx<double> *t1 = (Cx<double> *)ws, *t2 = (Cx<double> *)(ws + o2);
        PD_TRY_HIP(launch_admm_twiddle<double>(t1, n1, st));
        PD_TRY_HIP(launch_admm_twiddle<double>(t2, n2, st));
        PD_TRY_HIP(launch_fft2<double>((Cx<double> *)data, n1, n2, batch, t1, t2, inverse != 0, st));
    }
    return PD_OK;
}

// -------------------------------------------------------------- Algorithm 1 --
// Theta~ = sum_k A~_k B_k (Section 3.2, Algorithm 1; Section 5), FP64.  Per term:
// the circulant generators of A_k from one probe per band (Section 5.1), the
// threshold of A_k on the host from the generators (largest entry magnitude whose
// dropped part has Schur bound sqrt(||E||_1 ||E||_inf) <= eps_k = eta / (m ||v_k||_inf)),
// then, for batches of columns mu, B_k e_mu = Psi^* (v_k . Psi e_mu) and
// C_k e_mu = A~_k B_k e_mu accumulated over k, compacted to CSC.
namespace {

constexpr int DEC_BATCH = 256;

struct DecLayout {
    size_t ctx, X, T, Y, ACC, G, pos, cnt, base, bands, off, tcnt, roff, res, ent, total;
};

int dec_nbands(int L) { return 3 * L + 1; }

// Worst-case table sizes for m terms: every generator entry of a pair's block kept (each block
// covers one band, nb blocks per band: 2 nb N entries per term) and one residue class per source
// position of a coarser-target pair (at most nb N per term) plus two offsets per pair.
DecLayout dec_layout(const pd_shape *sh, int m = 1)
{
    const size_t N = (size_t)sh->n1 * sh->n2;
    const int nb = dec_nbands(sh->levels);
    const int P = (int)std::max<size_t>(std::min<size_t>(N, DEC_BATCH), (size_t)(2 * nb));
    pd_shape sc = *sh;
    sc.channels = P;
    DecLayout l;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    l.ctx = take(layout(&sc, 8).total);
    l.X = take((size_t)P * N * 8);
    l.T = take((size_t)P * N * 8);
    l.Y = take((size_t)P * N * 8);
    l.ACC = take((size_t)P * N * 8);
    l.G = take((size_t)2 * nb * N * 8);
    l.pos = take((size_t)2 * nb * 4);
    l.cnt = take((size_t)P * 8);
    l.base = take((size_t)P * 8);
    l.bands = take((size_t)nb * sizeof(DecBand));
    const size_t pairs = (size_t)m * nb * nb;
    l.off = take(pairs * 8);
    l.tcnt = take(pairs * 4);
    l.roff = take(pairs * 8);
    l.res = take(((size_t)m * nb * N + 2 * pairs) * 4);
    l.ent = take((size_t)m * 2 * nb * N * sizeof(DecEntry));
    l.total = off;
    return l;
}

std::vector<DecBand> dec_bands(int n1, int n2, int L)
{
    std::vector<DecBand> b;
    for (int lev = 1; lev <= L; ++lev) {
        const int g2 = n2 >> lev, g1 = n1 >> lev;
        b.push_back({lev, 0, g1, g2, g1});   // x1 high
        b.push_back({lev, g2, 0, g2, g1});   // x2 high
        b.push_back({lev, g2, g1, g2, g1});  // both high
    }
    b.push_back({L, 0, 0, n2 >> L, n1 >> L});  // approximation
    return b;
}

// Host side of the threshold: col[b'] / row[b] are the generator planes (Mallat layout) of A_k's
// column at source band b''s origin and of its row at target band b's origin.
struct DecGen {
    const std::vector<DecBand> &B;
    const double *col, *row;  // [nb][N]
    int n1;
    int64_t N;
    double at(const double *g, int which, const DecBand &b, int q2, int q1) const
    {
        return std::fabs(g[(int64_t)which * N + (int64_t)(b.o2 + q2) * n1 + b.o1 + q1]);
    }
    // max over columns and rows of the dropped magnitudes (|a| <= t), then the Schur bound
    double bound(double t) const
    {
        const int nb = (int)B.size();
        double colmax = 0.0, rowmax = 0.0;
        std::vector<double> tot, R;
        for (int side = 0; side < 2; ++side) {
            for (int x = 0; x < nb; ++x) {  // side 0: source band x (columns); side 1: target band x (rows)
                const int lx = B[x].lev;
                double base = 0.0;
                int F = 1;
                for (int y = 0; y < nb; ++y) {
                    const int ly = B[y].lev;
                    if (side == 0 ? ly > lx : ly >= lx) F = std::max(F, 1 << std::abs(ly - lx));
                }
                tot.assign((size_t)F * F, 0.0);
                for (int y = 0; y < nb; ++y) {
                    const int ly = B[y].lev;
                    // the block's generator and the band its entries lie in
                    const bool by_col = side == 0 ? ly <= lx : ly >= lx;
                    const double *g = by_col ? col : row;
                    const int which = side == 0 ? (by_col ? x : y) : (by_col ? y : x);
                    const DecBand &eb = side == 0 ? (by_col ? B[y] : B[x]) : (by_col ? B[x] : B[y]);
                    const bool residues = side == 0 ? ly > lx : ly >= lx;
                    if (!residues) {
                        for (int q2 = 0; q2 < eb.g2; ++q2)
                            for (int q1 = 0; q1 < eb.g1; ++q1) {
                                const double a = at(g, which, eb, q2, q1);
                                if (a <= t) base += a;
                            }
                        continue;
                    }
                    const int f = 1 << std::abs(ly - lx);
                    R.assign((size_t)f * f, 0.0);
                    for (int q2 = 0; q2 < eb.g2; ++q2)
                        for (int q1 = 0; q1 < eb.g1; ++q1) {
                            const double a = at(g, which, eb, q2, q1);
                            if (a <= t) R[(q2 % f) * f + (q1 % f)] += a;
                        }
                    for (int r2 = 0; r2 < F; ++r2)
                        for (int r1 = 0; r1 < F; ++r1) tot[(size_t)r2 * F + r1] += R[(r2 % f) * f + (r1 % f)];
                }
                double mx = 0.0;
                for (double v : tot) mx = std::max(mx, v);
                mx += base;
                if (side == 0)
                    colmax = std::max(colmax, mx);
                else
                    rowmax = std::max(rowmax, mx);
            }
        }
        return std::sqrt(colmax * rowmax);
    }
    // every entry magnitude of A_k (each block's generator over its band), nonzero, sorted, unique
    std::vector<double> candidates() const
    {
        const int nb = (int)B.size();
        std::vector<double> v;
        for (int bp = 0; bp < nb; ++bp)
            for (int b = 0; b < nb; ++b) {
                const bool by_col = B[b].lev <= B[bp].lev;
                const DecBand &eb = by_col ? B[b] : B[bp];
                for (int q2 = 0; q2 < eb.g2; ++q2)
                    for (int q1 = 0; q1 < eb.g1; ++q1) {
                        const double a = at(by_col ? col : row, by_col ? bp : b, eb, q2, q1);
                        if (a != 0.0) v.push_back(a);
                    }
            }
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        return v;
    }
};

int decompose_impl(const pd_shape *sh, const pd_operator *op, const pd_wavelet *wav, double eta, int64_t capacity,
                   int64_t *nnz_out, int64_t *col_ptr, int32_t *rows, double *vals, void *workspace,
                   size_t ws_bytes, hipStream_t st)
{
    const int n1 = sh->n1, n2 = sh->n2, L = sh->levels, m = op->terms, R = op->radius;
    const int64_t N = (int64_t)n1 * n2;
    const int nb = dec_nbands(L);
    const DecLayout Ly = dec_layout(sh, m);
    if (ws_bytes < Ly.total) return PD_ERR_WORKSPACE;
    char *ws = (char *)workspace;
    const int P = (int)std::max<int64_t>(std::min<int64_t>(N, DEC_BATCH), 2 * nb);
    double *X = (double *)(ws + Ly.X), *T = (double *)(ws + Ly.T), *Y = (double *)(ws + Ly.Y);
    double *ACC = (double *)(ws + Ly.ACC), *G = (double *)(ws + Ly.G);
    int *dpos = (int *)(ws + Ly.pos);
    int64_t *dcnt = (int64_t *)(ws + Ly.cnt), *dbase = (int64_t *)(ws + Ly.base);
    // host buffers that asynchronous copies read or write, and a join that runs before they are
    // destroyed on every return path (declared after them, so destroyed first)
    struct DecHost {
        std::vector<DecBand> bands;
        std::vector<int> pos, cnt, res;
        std::vector<double> hv, hga;
        std::vector<int64_t> off, roff, hc, hbase, cp;
        std::vector<DecEntry> ent;
    } H;
    struct StreamJoin {
        hipStream_t s;
        ~StreamJoin() { (void)hipStreamSynchronize(s); }
    } join{st};
    H.bands = dec_bands(n1, n2, L);
    const std::vector<DecBand> &bands = H.bands;
    PD_TRY_HIP(hipMemcpyAsync(ws + Ly.bands, bands.data(), nb * sizeof(DecBand), hipMemcpyHostToDevice, st));
    // probes: a Dirac at every band origin (columns, then rows)
    H.pos.assign(2 * nb, 0);
    std::vector<int> &pos = H.pos;
    for (int b = 0; b < nb; ++b) pos[b] = pos[nb + b] = bands[b].o2 * n1 + bands[b].o1;
    PD_TRY_HIP(hipMemcpyAsync(dpos, pos.data(), pos.size() * 4, hipMemcpyHostToDevice, st));
    // multipliers on the host for ||v_k||_inf
    H.hv.assign((size_t)m * N, 0.0);
    std::vector<double> &hv = H.hv;
    PD_TRY_HIP(hipMemcpyAsync(hv.data(), op->mult, hv.size() * 8, hipMemcpyDeviceToHost, st));
    pd_shape sc = *sh;
    sc.channels = 2 * nb;
    {
        Ctx<double> c = make_ctx<double>(&sc, wav, ws + Ly.ctx, st, 0);
        if (c.ts.nt > 0 && !c.tail) return PD_ERR_HIP;
        // generators of every term (probe transforms on the device), then the thresholds and
        // kept lists of the terms in parallel host threads, merged in term order
        H.hga.assign((size_t)m * 2 * nb * N, 0.0);
        std::vector<double> &hga = H.hga;
        for (int k = 0; k < m; ++k) {
            const double *uk = (const double *)op->taps + (int64_t)k * (2 * R + 1) * (2 * R + 1);
            PD_TRY_HIP(launch_dec_dirac_at(X, dpos, 2 * nb, N, st));
            int rc;
            if ((rc = synth_chain<double>(c, X, X, 0.0, T)) != PD_OK) return rc;
            PD_TRY_HIP(timed(PD_K_DECOMP, 0, st, [&] { return launch_dec_conv(T, X, nb, uk, R, n1, n2, 0, st); }));
            PD_TRY_HIP(timed(PD_K_DECOMP, 0, st, [&] {
                return launch_dec_conv(T + (int64_t)nb * N, X + (int64_t)nb * N, nb, uk, R, n1, n2, 1, st);
            }));
            if ((rc = analysis_plain<double>(c, X, G)) != PD_OK) return rc;
            PD_TRY_HIP(hipMemcpyAsync(hga.data() + (size_t)k * 2 * nb * N, G, (size_t)2 * nb * N * 8,
                                      hipMemcpyDeviceToHost, st));
        }
        PD_TRY_HIP(hipStreamSynchronize(st));
        struct Kept {
            std::vector<int64_t> off, roff;
            std::vector<int> cnt, res;
            std::vector<DecEntry> ent;
        };
        std::vector<Kept> kept(m);
        auto select = [&](int k) {
            const double *hg = hga.data() + (size_t)k * 2 * nb * N;
            double vinf = 0.0;
            for (int64_t i = 0; i < N; ++i) vinf = std::max(vinf, std::fabs(hv[(size_t)k * N + i]));
            DecGen gen{bands, hg, hg + (size_t)nb * N, n1, N};
            double t = 0.0;
            const bool keep_none = vinf == 0.0;  // V_k = 0: the term contributes nothing
            if (!keep_none) {
                const double eps = eta / ((double)m * vinf);
                const std::vector<double> cand = gen.candidates();
                int lo = 0, hi = (int)cand.size() - 1;
                while (lo <= hi) {  // the bound grows with t: bisect over the sorted magnitudes
                    const int mid = (lo + hi) / 2;
                    if (gen.bound(cand[mid]) <= eps) {
                        t = cand[mid];
                        lo = mid + 1;
                    } else {
                        hi = mid - 1;
                    }
                }
            }
            // kept generator entries per (source, target) pair; coarser targets grouped by residue
            Kept &K = kept[k];
            for (int bp = 0; bp < nb; ++bp)
                for (int b = 0; b < nb; ++b) {
                    const bool by_col = bands[b].lev <= bands[bp].lev;
                    const DecBand &eb = by_col ? bands[b] : bands[bp];
                    const double *g = by_col ? gen.col + (int64_t)bp * N : gen.row + (int64_t)b * N;
                    K.off.push_back((int64_t)K.ent.size());
                    K.roff.push_back((int64_t)K.res.size());
                    const int f = by_col ? 1 : 1 << (bands[b].lev - bands[bp].lev);
                    std::vector<std::vector<DecEntry>> cls((size_t)f * f);
                    if (!keep_none)
                        for (int q2 = 0; q2 < eb.g2; ++q2)
                            for (int q1 = 0; q1 < eb.g1; ++q1) {
                                const double a = g[(int64_t)(eb.o2 + q2) * n1 + eb.o1 + q1];
                                if (std::fabs(a) > t) cls[(q2 % f) * f + (q1 % f)].push_back({q2, q1, a});
                            }
                    int run = 0;
                    for (auto &v : cls) {
                        K.res.push_back(run);
                        K.ent.insert(K.ent.end(), v.begin(), v.end());
                        run += (int)v.size();
                    }
                    K.res.push_back(run);
                    K.cnt.push_back(run);
                }
        };
        {
            std::vector<std::thread> pool;
            for (int k = 1; k < m; ++k) pool.emplace_back(select, k);
            select(0);
            for (auto &th : pool) th.join();
        }
        std::vector<int64_t> &off = H.off, &roff = H.roff;
        std::vector<int> &cnt = H.cnt, &res = H.res;
        std::vector<DecEntry> &ent = H.ent;
        for (int k = 0; k < m; ++k) {
            const int64_t eb = (int64_t)ent.size(), rb = (int64_t)res.size();
            for (int64_t o : kept[k].off) off.push_back(eb + o);
            for (int64_t o : kept[k].roff) roff.push_back(rb + o);
            cnt.insert(cnt.end(), kept[k].cnt.begin(), kept[k].cnt.end());
            res.insert(res.end(), kept[k].res.begin(), kept[k].res.end());
            ent.insert(ent.end(), kept[k].ent.begin(), kept[k].ent.end());
        }
        // the tables, in the workspace (sized for the worst case)
        if (res.size() * 4 > Ly.ent - Ly.res || ent.size() * sizeof(DecEntry) > Ly.total - Ly.ent) return PD_ERR_HIP;
        DecTables tb{};
        tb.nb = nb;
        tb.n1 = n1;
        tb.n2 = n2;
        tb.bands = (const DecBand *)(ws + Ly.bands);
        tb.off = (const int64_t *)(ws + Ly.off);
        tb.cnt = (const int *)(ws + Ly.tcnt);
        tb.roff = (const int64_t *)(ws + Ly.roff);
        tb.res = (const int *)(ws + Ly.res);
        tb.ent = (const DecEntry *)(ws + Ly.ent);
        PD_TRY_HIP(hipMemcpyAsync(ws + Ly.off, off.data(), off.size() * 8, hipMemcpyHostToDevice, st));
        PD_TRY_HIP(hipMemcpyAsync(ws + Ly.tcnt, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, st));
        PD_TRY_HIP(hipMemcpyAsync(ws + Ly.roff, roff.data(), roff.size() * 8, hipMemcpyHostToDevice, st));
        PD_TRY_HIP(hipMemcpyAsync(ws + Ly.res, res.data(), res.size() * 4, hipMemcpyHostToDevice, st));
        if (!ent.empty())
            PD_TRY_HIP(hipMemcpyAsync(ws + Ly.ent, ent.data(), ent.size() * sizeof(DecEntry), hipMemcpyHostToDevice, st));
        {
            // columns in batches of P
            pd_shape sb = *sh;
            sb.channels = P;
            Ctx<double> cb = make_ctx<double>(&sb, wav, ws + Ly.ctx, st, 0);
            if (cb.ts.nt > 0 && !cb.tail) return PD_ERR_HIP;
            H.hc.assign(P, 0);
            H.hbase.assign(P, 0);
            H.cp.assign((size_t)N + 1, 0);
            std::vector<int64_t> &hc = H.hc, &hbase = H.hbase, &cp = H.cp;
            int64_t total = 0;
            for (int64_t j0 = 0; j0 < N; j0 += P) {
                const int np = (int)std::min<int64_t>(P, N - j0);
                int r;
                PD_TRY_HIP(launch_dec_dirac(T, j0, P, N, st));
                if ((r = synth_chain<double>(cb, T, T, 0.0, X)) != PD_OK) return r;  // psi_mu
                PD_TRY_HIP(launch_fill<double>(ACC, 0.0, (int64_t)P * N, st));
                for (int k = 0; k < m; ++k) {
                    PD_TRY_HIP(timed(PD_K_DECOMP, 1, st, [&] {
                        return launch_dec_mul(X, (const double *)op->mult + (int64_t)k * N, T, P, N, st);
                    }));
                    if ((r = analysis_plain<double>(cb, T, Y)) != PD_OK) return r;  // B_k e_mu
                    PD_TRY_HIP(timed(PD_K_DECOMP, 2, st, [&] { return launch_dec_acc(Y, ACC, np, tb, k, st); }));
                }
                PD_TRY_HIP(timed(PD_K_DECOMP, 3, st, [&] { return launch_dec_count(ACC, np, N, dcnt, st); }));
                PD_TRY_HIP(hipMemcpyAsync(hc.data(), dcnt, np * 8, hipMemcpyDeviceToHost, st));
                PD_TRY_HIP(hipStreamSynchronize(st));
                for (int j = 0; j < np; ++j) {
                    hbase[j] = total;
                    total += hc[j];
                    cp[(size_t)(j0 + j) + 1] = total;
                }
                if (total <= capacity && rows && vals) {
                    PD_TRY_HIP(hipMemcpyAsync(dbase, hbase.data(), np * 8, hipMemcpyHostToDevice, st));
                    PD_TRY_HIP(
                        timed(PD_K_DECOMP, 4, st, [&] { return launch_dec_fill(ACC, np, N, dbase, rows, vals, st); }));
                    PD_TRY_HIP(hipStreamSynchronize(st));  // hbase is rewritten by the next batch
                }
            }
            *nnz_out = total;
            PD_TRY_HIP(hipMemcpyAsync(col_ptr, cp.data(), cp.size() * 8, hipMemcpyHostToDevice, st));
            PD_TRY_HIP(hipStreamSynchronize(st));  // the host tables and cp live until here
            return total <= capacity ? PD_OK : PD_ERR_WORKSPACE;
        }
    }
}

}  // namespace

extern "C" size_t pd_decompose_workspace_size(const pd_shape *shape, int32_t terms)
{
    if (!shape || shape->levels < 1 || terms < 1 || terms > PD_MAX_PC) return 0;
    pd_shape s = *shape;
    s.channels = 1;
    if (check_shape(&s) != PD_OK) return 0;
    return dec_layout(&s, terms).total;
}

extern "C" int pd_decompose(const pd_shape *shape, const pd_operator *op, const pd_wavelet *wav, double eta,
                            int64_t capacity, int64_t *nnz, int64_t *col_ptr, int32_t *rows, double *vals,
                            void *workspace, size_t ws_bytes, void *stream)
{
    int rc;
    if (!shape) return PD_ERR_ARG;
    pd_shape s = *shape;
    if (s.channels != 1) return PD_ERR_SHAPE;
    if ((rc = check_shape(&s)) || (rc = check_op(op, &s)) || (rc = check_wavelet(wav))) return rc;
    if (s.levels < 1) return PD_ERR_SHAPE;
    if (op->kind != PD_OP_PC) return PD_ERR_UNSUPPORTED;
    if (!std::isfinite(eta) || eta < 0.0) return PD_ERR_TAU;
    if (!nnz || !col_ptr || !workspace || capacity < 0 || (capacity > 0 && (!rows || !vals))) return PD_ERR_ARG;
    if ((int64_t)s.n1 * s.n2 > INT32_MAX) return PD_ERR_UNSUPPORTED;
    return decompose_impl(&s, op, wav, eta, capacity, nnz, col_ptr, rows, vals, workspace, ws_bytes,
                          (hipStream_t)stream);
}
