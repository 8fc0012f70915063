/*
 * pd.h -- C ABI of libpd, an MI355X (gfx950) solver for the wavelet-l1
 * deblurring energy of Escande & Weiss, "Fast Wavelet Decomposition of Linear
 * Operators through Product-Convolution Expansions" (arXiv:2005.09870):
 *
 *     argmin_f  E(f) = 1/2 ||H f - f0||_2^2 + ||Psi^* f||_{1,w}          (eq. 4.1)
 *
 * solved in coefficient form (Appendix A.1, eq. A.1) by FISTA with the exact
 * spatial operator ("FISTA-Spa", Table 1):
 *
 *     z(0) = y(1) = init
 *     z(i)   = Prox_{tau ||.||_{1,w}}( y(i) - tau Psi^* H^T (H Psi y(i) - f0) )
 *     y(i+1) = z(i) + (i-1)/(i+2) (z(i) - z(i-1))
 *
 * Psi is a periodic orthogonal separable 2-D wavelet transform (Sections 2.1,
 * 2.2); H is a row-separable spatially varying blur whose impulse response
 * depends on the source row only (Operator 1 of Section 4.1 is one).
 *
 * Conventions for every entry point
 *  - Images and coefficient planes are row-major, x1 (index i1) fastest:
 *    element (c, i2, i1) of a C x n2 x n1 planar array is at c*n1*n2 + i2*n1 + i1.
 *  - Wavelet coefficients use the Mallat layout in an n2 x n1 plane: after one
 *    level the band low-pass in both axes is at [0,n2/2) x [0,n1/2), the band
 *    high-pass along x1 at [0,n2/2) x [n1/2,n1), high-pass along x2 at
 *    [n2/2,n2) x [0,n1/2), high-pass in both at [n2/2,n2) x [n1/2,n1); the next
 *    level recurses on the first band.
 *  - Band index k (weights): k = 0 is the coarsest approximation band, k = 1..L
 *    the detail bands from the coarsest (decomposition level L) to the finest
 *    (level 1).  For a full-depth transform k - 1 is the paper's scale |lambda|.
 *  - "device" pointers are HIP device memory owned by the caller; libpd never
 *    allocates or frees device memory: scratch space comes from a caller
 *    workspace of the size the matching *_workspace_size call reports.
 *    "host" pointers are read during the call only.
 *  - Every GPU entry point enqueues its work on `stream` (a hipStream_t; NULL
 *    is the default stream) and returns without synchronising unless stated.
 *  - Every entry point returns PD_OK (0) or a negative pd_status; nothing is
 *    thrown across the ABI.  On an argument error nothing is enqueued.
 *  - Element type of every device array is the call's dtype (float or double).
 *  - Concurrent calls that share a workspace race; distinct workspaces are
 *    independent.
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PD_OK = 0,
    PD_ERR_ARG = -1,         /* null pointer, bad enum, negative count          */
    PD_ERR_SHAPE = -2,       /* n1 or n2 not divisible by 2^levels, bad sizes   */
    PD_ERR_WORKSPACE = -3,   /* workspace smaller than required                 */
    PD_ERR_TAU = -4,         /* step size <= 0 or not finite                    */
    PD_ERR_NONFINITE = -5,   /* a prox argument was NaN/Inf (check_finite only) */
    PD_ERR_HIP = -6,         /* a HIP runtime call failed                       */
    PD_ERR_UNSUPPORTED = -7  /* valid request outside what libpd supports       */
} pd_status;

typedef enum { PD_F32 = 0, PD_F64 = 1 } pd_dtype;

typedef enum {
    PD_OP_IDENTITY = 0, /* H = Id: wavelet denoising, the closed-form special case      */
    PD_OP_ROWBLUR = 1,  /* H f(x) = sum_y k_{y2}(x1-y1) k_{y2}(x2-y2) f(y), periodic:     */
                        /* the response of source row y2 is the outer product of one    */
                        /* 1-D profile k_{y2}[-R..R] with itself (Section 1, eq. 1.1;   */
                        /* Operator 1 of Section 4.1 when built by pd_op1_taps)         */
    PD_OP_PC = 2        /* product-convolution expansion (Section 1, Section 3.1; the   */
                        /* operator of FISTA-PC, Table 1):                              */
                        /*   H f = sum_{k<m} u_k * (v_k . f),                           */
                        /*   (u * g)(x) = sum_d u(d) g(x - d), d in [-R, R]^2, periodic */
} pd_op_kind;

/* Problem size: n1 x n2 pixels (n1 fastest), `channels` planar channels,
 * `levels` >= 1 decomposition levels; n1 and n2 must be divisible by
 * 2^levels, levels <= 16, channels in [1, 4]. */
typedef struct {
    int32_t n1, n2, channels, levels;
} pd_shape;

/* Blur operator, radius in [0, 9].
 *   PD_OP_ROWBLUR: taps = device array [n2][2*radius+1] of the call's dtype,
 *     row i2 holding the profile k_{i2}[d], d = -radius..radius, of SOURCE
 *     row i2; terms and mult unused.
 *   PD_OP_PC: terms = m in [1, 64]; taps = device [m][2*radius+1][2*radius+1]
 *     kernels u_k, row-major in (d2, d1) with d = -radius..radius; mult =
 *     device [m][n2][n1] multipliers v_k, shared by the channels.  Supported
 *     by pd_solve and pd_apply_op (not pd_solve_batched or pd_backward:
 *     PD_ERR_UNSUPPORTED).
 *   PD_OP_IDENTITY: all fields unused. */
typedef struct {
    int32_t kind;
    int32_t radius;
    const void *taps;
    int32_t terms;
    const void *mult;
} pd_operator;

/* Low-pass filter h[0..len-1] of the orthogonal wavelet (Section 2.1; the
 * high-pass filter is derived as g[k] = (-1)^(1-k) h[1-k]).  host doubles;
 * len even, 2 <= len <= 12 (12 = Symmlet of order 6, Section 4.2). */
typedef struct {
    int32_t len;
    const double *h;
} pd_wavelet;

/* Weights w of the weighted l1 norm (eq. 4.1).  Exactly one of
 *   level_w : host doubles [levels+1], one weight per band index k, or
 *   coeff_w : device array [channels][n2][n1] (Mallat layout), one weight per
 *             coefficient,
 * is non-NULL.  joint != 0 selects group soft-thresholding of the channel
 * vector of each coefficient (an extension for colour images, not in the
 * paper; level_w only). */
typedef struct {
    const double *level_w;
    const void *coeff_w;
    int32_t joint;
} pd_weights;

/* Iteration parameters.  tau > 0 is the step (the paper asks tau <=
 * ||H||^-2).  iters >= 0 iterations are run, numbered iter_offset+1 ..
 * iter_offset+iters (the momentum uses the global number).  check_finite != 0
 * makes the call synchronise the stream at the end and return
 * PD_ERR_NONFINITE if any prox argument was not finite. */
typedef struct {
    double tau;
    int32_t iters;
    int32_t iter_offset;
    int32_t check_finite;
} pd_params;

/* Bytes of device workspace pd_solve needs for this size and dtype. */
size_t pd_workspace_size(const pd_shape *shape, int32_t dtype);

/* Run FISTA on eq. 4.1 (Appendix A.1).
 *   f0      device [C][n2][n1] observation.
 *   z_cur, z_prev  device [C][n2][n1] Mallat coefficient state, in/out.  On
 *           entry they hold z(k) and z(k-1) for k = iter_offset (for k = 0 both
 *           hold z(0)); on exit z(k+iters) and z(k+iters-1).  If init_from_f0
 *           != 0 both are first set to Psi^* f0 (the default initial guess).
 *   f_out   device [C][n2][n1] or NULL: receives Psi z(k+iters).
 *   stats   device double [iters][3] or NULL: for each iteration i, the two
 *           terms of eq. 4.1 at y(i), 1/2||H Psi y(i) - f0||^2 and
 *           ||y(i)||_{1,w}, and ||z(i) - y(i)||^2 (the squared gradient-mapping
 *           norm times tau^2).  Accumulated in FP64; the caller zeroes it.
 * Errors: PD_ERR_ARG, PD_ERR_SHAPE, PD_ERR_TAU, PD_ERR_WORKSPACE,
 * PD_ERR_UNSUPPORTED, PD_ERR_HIP, PD_ERR_NONFINITE (check_finite only). */
int pd_solve(const pd_shape *shape, int32_t dtype, const pd_operator *op,
             const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
             const void *f0, void *z_cur, void *z_prev, int32_t init_from_f0,
             void *f_out, double *stats, void *workspace, size_t ws_bytes,
             void *stream);

/* Scratch bytes pd_solve_noalloc holds per GPU: pd_workspace_size of the
 * problem must not exceed it (16 MiB: e.g. 1024 x 1024 FP32 with one channel,
 * 512 x 512 with up to 4 channels, or 512 x 512 FP64). */
#define PD_NOALLOC_SCRATCH_BYTES (16u << 20)

/* pd_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments without the workspace, the same results bit for bit.  Its
 * scratch is a fixed device array of PD_NOALLOC_SCRATCH_BYTES inside the
 * library (one per GPU, held until the process ends); the call allocates
 * nothing and does not replay graphs (every iteration is launched).  Every
 * call on one GPU shares that array and leaves its contents behind (the
 * call clears what it needs cleared), so calls that overlap on one GPU --
 * from several threads or on several streams -- race.  A problem whose
 * pd_workspace_size exceeds PD_NOALLOC_SCRATCH_BYTES is rejected with
 * PD_ERR_WORKSPACE before anything is enqueued.  Other errors as pd_solve. */
int pd_solve_noalloc(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                     const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                     const void *f0, void *z_cur, void *z_prev, int32_t init_from_f0,
                     void *f_out, double *stats, void *stream);

/* One image of a batch for pd_solve_batched.  Arrays of image b start at
 * element `offset` of the packed buffers (each image planar C x n2 x n1).
 * op: PD_OP_ROWBLUR with the image's own device tap table.  w: the image's
 * weights as for pd_solve (host level_w, or coeff_w = the image's own device
 * [C][n2][n1] map; joint = group prox over its channels). */
typedef struct {
    pd_shape shape;
    int64_t offset;
    double tau;
    pd_operator op;
    pd_weights w;
} pd_image_desc;

/* Bytes of device workspace pd_solve_batched needs for these images. */
size_t pd_batched_workspace_size(int32_t batch, const pd_image_desc *descs, int32_t dtype);

/* Solve `batch` independent instances of eq. 4.1 of uneven sizes from the
 * default initial guess, `iters` iterations each, in lock-step launches that
 * cover every image (the same per-image arithmetic as pd_solve, so results
 * match pd_solve bit for bit).  f0_packed / f_out_packed: device, packed
 * back to back in order as described by descs[b].offset.  stats: device
 * double [batch][iters][3] or NULL (caller-zeroed, as for pd_solve).  descs
 * is a host array, read during the call.  Every image of a batch takes the
 * same prox: all scalar, or all joint with one channel count (else
 * PD_ERR_UNSUPPORTED).  The per-image descriptor tables are copied into the
 * workspace through a library-owned pinned staging buffer, so the call
 * returns without synchronising the host.  The iterations between the first
 * and the last run in replayed graph chunks as for pd_solve (pd_graphs_enable),
 * with bitwise the same results.  Errors as pd_solve. */
int pd_solve_batched(int32_t batch, const pd_image_desc *descs, int32_t dtype,
                     const pd_wavelet *wav, int32_t iters, const void *f0_packed,
                     void *f_out_packed, double *stats, void *workspace,
                     size_t ws_bytes, void *stream);

/* Bytes of device workspace pd_backward needs. */
size_t pd_backward_workspace_size(const pd_shape *shape, int32_t dtype, int32_t iters,
                                  int32_t checkpoint_every);

/* Reverse mode of pd_solve from the default initial guess (init = Psi^* f0,
 * iter_offset = 0, scalar prox), for f = Psi z(iters):
 *   grad_f   device [C][n2][n1]: dLoss/df.
 *   grad_f0  device [C][n2][n1] or NULL: receives dLoss/df0.
 *   grad_w   device [C][n2][n1] or NULL: receives dLoss/dw (needs coeff_w).
 * The forward recursion is recomputed internally in segments of
 * `checkpoint_every` iterations from stored (z(i), z(i-1)) pairs, so memory
 * is O(iters/checkpoint_every + checkpoint_every) planes.  The derivative of
 * the soft threshold at the kink |v| = tau w is taken as 0.
 * Errors as pd_solve. */
int pd_backward(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                const void *f0, const void *grad_f, void *grad_f0, void *grad_w,
                int32_t checkpoint_every, void *workspace, size_t ws_bytes,
                void *stream);

/* Forward solve that keeps what pd_backward needs: from the default initial
 * guess, `prm->iters` iterations (iter_offset = 0, scalar prox) with
 * (z(i), z(i-1)) stored at the start of every segment of `checkpoint_every`
 * iterations in `workspace` (pd_backward_workspace_size bytes), and
 * f_out (device [C][n2][n1]) = Psi z(iters), bitwise the f of pd_solve.  A
 * following pd_backward_checkpointed with the same arguments and workspace
 * then skips its own forward pass.  Errors as pd_backward. */
int pd_solve_checkpointed(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                          const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                          const void *f0, void *f_out, int32_t checkpoint_every, void *workspace,
                          size_t ws_bytes, void *stream);

/* pd_backward reading the checkpoints that pd_solve_checkpointed stored in
 * `workspace` (same shape, operator, weights, parameters and f0; the
 * workspace untouched in between) instead of recomputing them: the same
 * gradients bit for bit, one forward pass less.  The checkpoints are only
 * read, so it may be called again for another grad_f.  Errors as pd_backward. */
int pd_backward_checkpointed(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                             const pd_wavelet *wav, const pd_weights *w, const pd_params *prm,
                             const void *f0, const void *grad_f, void *grad_f0, void *grad_w,
                             int32_t checkpoint_every, void *workspace, size_t ws_bytes,
                             void *stream);

/* Building blocks, exposed for tests and for setting up a solve.            */

/* Forward (inverse == 0: out = Psi^* in) or inverse (out = Psi in) periodic
 * 2-D wavelet transform of C channels (Sections 2.1-2.2).  in and out are
 * device [C][n2][n1] and must not overlap.  workspace: pd_workspace_size bytes. */
int pd_fwt(const pd_shape *shape, int32_t dtype, const pd_wavelet *wav,
           int32_t inverse, const void *in, void *out, void *workspace,
           size_t ws_bytes, void *stream);

/* out = H in (transpose == 0) or H^T in (transpose != 0) for C channels;
 * device [C][n2][n1], non-overlapping. */
int pd_apply_op(const pd_shape *shape, int32_t dtype, const pd_operator *op,
                int32_t transpose, const void *in, void *out, void *stream);

/* Autotuning of the blur.  Times its variants for this size and operator on
 * the caller's stream and records the fastest in a process-wide cache keyed
 * by (n1, n2, channels, radius, dtype), which pd_solve, pd_solve_noalloc,
 * pd_solve_checkpointed and pd_backward use from then on (variant 32 for
 * sizes never tuned).  Variants (PD_BLUR_* codes): 32 and 48 = one fused
 * kernel with that many output rows per workgroup; 1020, 1039 and 1058 = two
 * kernels (r = H x - f0, then s = H^T r) whose waves walk down strips of
 * 128 columns in blocks of 20, 39 or 58 rows.  Every variant computes each
 * output by the same sums in the same order, so results do not depend on the
 * choice.  workspace: at least pd_workspace_size bytes, used as scratch.
 * chosen (host, nullable): if it holds one of the codes on entry, that
 * variant is recorded without timing; on return it holds the recorded code
 * (0 for operators with no variants).  Synchronises the host with `stream`
 * when timing.  Errors: PD_ERR_ARG, PD_ERR_SHAPE, PD_ERR_WORKSPACE,
 * PD_ERR_UNSUPPORTED, PD_ERR_HIP. */
#define PD_BLUR_TILE32 32
#define PD_BLUR_TILE48 48
#define PD_BLUR_SPLIT20 1020
#define PD_BLUR_SPLIT39 1039
#define PD_BLUR_SPLIT58 1058
int pd_tune(const pd_shape *shape, int32_t dtype, const pd_operator *op, void *workspace,
            size_t ws_bytes, int32_t *chosen, void *stream);

/* Host: low-pass filter of the orthogonal wavelet with `moments` vanishing
 * moments and minimal support 2*moments whose phase is closest to linear
 * (the Symmlet family; Section 2.1 filter bank, Section 4.2 "Symmlet of order
 * 6"), normalised to sum sqrt(2).  h_out: host double [2*moments].
 * moments in [1, 10]. */
int pd_symmlet(int32_t moments, double *h_out);

/* Host: Operator 1 of Section 4.1.  Source row i2 emits an isotropic Gaussian
 * of standard deviation sigma_max * i2/(n2-1) pixels, truncated to the square
 * window that keeps the fraction `mass` of the Gaussian and renormalised to
 * unit sum.  Writes the common half-width to *radius and, if taps_out is not
 * NULL, the profiles as host doubles [n2][2*radius+1]. */
int pd_op1_taps(int32_t n2, double sigma_max, double mass, int32_t *radius,
                double *taps_out);

/* Host: rank-`terms` product-convolution expansion H ~ sum_k u_k * (v_k . x)
 * of Operator 1 (Section 3.3.3): a randomized SVD of its space-varying impulse
 * response S, which has one row per window offset (d2, d1), row-major over
 * [-R, R]^2, and one column per source row y (the response of Operator 1
 * depends on the source row only): S[(d2, d1), y] = taps[y][d2+R] taps[y][d1+R].
 * The range of S is sampled with terms + oversample Gaussian vectors (a
 * SplitMix64 stream of `seed`, Box-Muller), refined by power_iters rounds of
 * subspace iteration and the projected matrix is decomposed exactly (one-sided
 * Jacobi); only products with S and S^T are formed.
 *   taps        host double [n2][2R+1], e.g. from pd_op1_taps; R = radius <= 64
 *   terms       requested rank, >= 1; oversample in [0, 64]; power_iters in [0, 16]
 *   u_out       host double [terms][(2R+1)^2]: orthonormal kernels, each with its
 *               entry of largest magnitude positive
 *   v_out       host double [terms][n2]: v_k(y) = <S(., y), u_k>, the multiplier
 *               of source row y (the same for every column of the row)
 *   sv_out      host double [terms] singular values, descending (may be NULL)
 *   terms_out   the rank produced: at most terms, terms + oversample, n2 and
 *               (2R+1)^2, and only singular values above 1e-14 of the largest
 * Returns PD_ERR_ARG for bad arguments or S = 0; never touches the GPU. */
int pd_pc_expansion(const double *taps, int32_t n2, int32_t radius, int32_t terms,
                    int32_t oversample, int32_t power_iters, uint64_t seed,
                    double *u_out, double *v_out, double *sv_out, int32_t *terms_out);

/* ---------------------------------------------------------------------------
 * FISTA in the wavelet domain (Section 4.3, eq. 4.3, and Appendix A.1).
 * Eq. 4.1 approximated as
 *
 *     argmin_z  1/2 ||Theta_L z - z0||^2 + ||z||_{1,w},   z0 = Psi^* f0,
 *
 * with Theta_L a sparse approximation of Theta = Psi^* H Psi given by the
 * caller, solved by
 *
 *     z(i)   = Prox^Sigma_{tau ||.||_{1,w}}( y(i) - tau Sigma Theta_L^T (Theta_L y(i) - z0) )
 *     y(i+1) = z(i) + (i-1)/(i+2) (z(i) - z(i-1))
 *
 * with Sigma = Id ("FISTA-W") or the Jacobi preconditioner ("FISTA-WP",
 * sigma_l = 1 / (Theta_L^T Theta_L)[l,l], 1 for an empty column of Theta_L).
 * Prox^Sigma is the prox in the metric of Sigma^{-1}: soft-thresholding of
 * coefficient l at tau * sigma_l * w_l.  One iteration is two sparse
 * products (with Theta_L and with its transpose, stored as its own CSR).
 * ------------------------------------------------------------------------- */

/* A square sparse matrix in CSR form, all arrays device memory:
 *   row_ptr int64 [n+1], row_ptr[0] = 0, nondecreasing, row_ptr[n] = nnz;
 *   col     int32 [nnz], the column indices of each row strictly increasing
 *           and in [0, n);
 *   val     [nnz] of the call's dtype.
 * Rows and columns of Theta_L are indexed by Mallat position i2*n1 + i1.
 * pd_csr_transpose checks these rules; the products do not, but they clamp
 * row bounds to [0, nnz] and columns to [0, n), so a malformed matrix gives
 * meaningless results without any access outside its arrays. */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const void *val;
} pd_csr;

/* Bytes of device workspace pd_csr_transpose needs for an n x n matrix. */
size_t pd_csr_transpose_workspace_size(int32_t n);

/* The transpose of a (set-up, not the iteration): t_row_ptr device int64
 * [n+1], t_col device int32 [nnz], t_val device [nnz], each row's columns
 * sorted, so the result does not depend on the order of atomic updates.
 * Checks a first and returns PD_ERR_ARG if it breaks the pd_csr rules; this
 * check synchronises the stream.  Errors: PD_ERR_ARG, PD_ERR_WORKSPACE,
 * PD_ERR_HIP. */
int pd_csr_transpose(const pd_csr *a, int32_t dtype, int64_t *t_row_ptr, int32_t *t_col,
                     void *t_val, void *workspace, size_t ws_bytes, void *stream);

/* y = a x (device [n] vectors, non-overlapping).  Errors: PD_ERR_ARG, PD_ERR_HIP. */
int pd_spmv(const pd_csr *a, int32_t dtype, const void *x, void *y, void *stream);

/* sigma (device [n]) = the Jacobi preconditioner of FISTA-WP from the
 * transpose theta_t = Theta_L^T: sigma_l = 1 / sum_k theta_t[l,k]^2, or 1
 * where that sum is 0.  Errors: PD_ERR_ARG, PD_ERR_HIP. */
int pd_wjacobi(const pd_csr *theta_t, int32_t dtype, void *sigma, void *stream);

/* Bytes of device workspace pd_wsolve needs (shape: channels = 1). */
size_t pd_wsolve_workspace_size(const pd_shape *shape, int32_t dtype);

/* Run FISTA-W (precond == 0) or FISTA-WP (precond != 0) on the problem above.
 *   shape   n1 x n2 Mallat plane, channels = 1, levels (for level_w bands).
 *   theta, theta_t  Theta_L and its transpose (pd_csr_transpose), n = n1*n2.
 *   w       level_w (host, bands as for pd_solve) or coeff_w (device [n]);
 *           joint must be 0.
 *   prm     tau > 0 (the step bound is 1/||Sigma^{1/2} Theta_L^T Theta_L
 *           Sigma^{1/2}||), iters, iter_offset (resume), check_finite.
 *   z0      device [n]: Psi^* f0 (pd_fwt).
 *   z_cur, z_prev  device [n] state, in/out, as for pd_solve: z(k), z(k-1)
 *           on entry (k = iter_offset), z(k+iters), z(k+iters-1) on exit; if
 *           init_from_z0 != 0 both are first set to z0.  f = Psi z_cur by pd_fwt.
 *   stats   device double [iters][3] or NULL: per iteration i,
 *           1/2||Theta_L y(i) - z0||^2, ||y(i)||_{1,w}, ||z(i) - y(i)||^2,
 *           accumulated in FP64; the caller zeroes it.
 * Errors: PD_ERR_ARG, PD_ERR_SHAPE, PD_ERR_TAU, PD_ERR_WORKSPACE,
 * PD_ERR_UNSUPPORTED, PD_ERR_HIP, PD_ERR_NONFINITE (check_finite only). */
int pd_wsolve(const pd_shape *shape, int32_t dtype, const pd_csr *theta, const pd_csr *theta_t,
              const pd_weights *w, const pd_params *prm, int32_t precond, const void *z0,
              void *z_cur, void *z_prev, int32_t init_from_z0, double *stats, void *workspace,
              size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------- ADMM-PC --
 * ADMM on eq. 4.1 with a product-convolution operator H = sum_k u_k * (v_k . f)
 * (Appendix A.2; Table 1).  With g = V f, z = Psi^* f and D = diag(gamma_k Id),
 * one iteration is, in this order,
 *   g  <- (U^T U + beta D)^-1 (U^T f0 - xi + beta D V f)
 *   z  <- Prox_{||.||_{1,w}/beta}(Psi^* f - zeta / beta)
 *   f  <- (beta sum_k gamma_k v_k^2 + beta)^-1 (V^T (xi + beta D g) + Psi (beta z + zeta))
 *   xi <- xi + beta D (g - V f);   zeta <- zeta + beta (z - Psi^* f),
 * started from f = f0, z = Psi^* f0, xi = zeta = 0.  The g system is solved
 * by the Woodbury identity, whose middle matrix Id + sum_k U_k U_k^T / (beta
 * gamma_k) is diagonal in the Fourier basis (periodic boundaries, 2-D FFTs);
 * gamma_k = max |u_k^| normalised to sum 1 (1/m if every kernel is 0).     */

/* Bytes of device workspace pd_admm_solve needs for m = terms. 0 on bad
 * arguments. */
size_t pd_admm_workspace_size(const pd_shape *shape, int32_t dtype, int32_t terms);

/* Run `iters` ADMM-PC iterations on each channel (the same operator).
 *   shape   n1 x n2 x channels, levels; n1 and n2 powers of two in [2, 4096]
 *           (FP32) or [2, 2048] (FP64), else PD_ERR_UNSUPPORTED.
 *   op      kind PD_OP_PC (taps [m][2R+1][2R+1], mult [m][n2][n1], device, in the dtype).
 *   w       level_w (host) or coeff_w (device [n2][n1], every channel);
 *           joint must be 0.
 *   beta    beta1 = beta2 > 0 (finite).
 *   f0      device [channels][n2][n1]; f_out, z_out device, same size,
 *           written (f and z after the last iteration; iters = 0 gives f0
 *           and Psi^* f0).  No two of f0, f_out, z_out may alias.
 *   stats   device double [iters][3] or NULL: per iteration, summed over
 *           channels, ||g - V f||^2_D, ||z - Psi^* f||^2 and ||z||_{1,w}
 *           (the primal residuals after the multiplier step, and the
 *           penalty), accumulated in FP64; zeroed by the call.
 * Asynchronous on `stream` (no host synchronisation).  Part of each iteration
 * (the transforms and the zeta / z step) runs on a library-owned second
 * stream of the current device, ordered by events against `stream` and joined
 * back into it before the call returns; calls that share a workspace on
 * different streams race, as for every entry point.
 * Errors: PD_ERR_ARG, PD_ERR_SHAPE, PD_ERR_TAU (beta), PD_ERR_WORKSPACE,
 * PD_ERR_UNSUPPORTED, PD_ERR_HIP. */
int pd_admm_solve(const pd_shape *shape, int32_t dtype, const pd_operator *op, const pd_wavelet *wav,
                  const pd_weights *w, double beta, int32_t iters, const void *f0, void *f_out, void *z_out,
                  double *stats, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of twiddle workspace pd_fft2 needs. 0 on bad arguments. */
size_t pd_fft2_workspace_size(int32_t n1, int32_t n2, int32_t dtype);

/* In-place 2-D DFT of `batch` complex planes (the transform ADMM-PC's g-update
 * uses): data device [batch][n2][n1] interleaved (re, im) of the dtype;
 * forward X(k) = sum_p x(p) exp(-2 pi i <k, p / n>), inverse with the opposite
 * sign and a 1/(n1 n2) scale.  Sizes as for pd_admm_solve.
 * Errors: PD_ERR_ARG, PD_ERR_WORKSPACE, PD_ERR_UNSUPPORTED, PD_ERR_HIP. */
int pd_fft2(int32_t n1, int32_t n2, int32_t batch, int32_t dtype, int32_t inverse, void *data, void *workspace,
            size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ Algorithm 1 --
 * The wavelet representation of a product-convolution operator H = sum_k U_k V_k
 * (Section 3.2, Algorithm 1; Section 5): Theta~ = sum_k A~_k B_k with
 * A_k = Psi^* U_k Psi, B_k = Psi^* V_k Psi, eps_k = eta / (m ||v_k||_inf) and A~_k
 * the entries of A_k above t_k, the largest entry magnitude whose dropped part E
 * has Schur bound sqrt(||E||_1 ||E||_inf) <= eps_k; then ||Theta - Theta~||_2 <= eta.
 * FP64 throughout.  A_k is formed from its circulant sub-band generators (one probe
 * transform per band and direction), B_k column by column, C_k = A~_k B_k by
 * spreading each nonzero of a column of B_k over the kept generator entries. */

/* Bytes of device workspace pd_decompose needs for m = terms (channels ignored).
 * Includes worst-case room for the kept generator entries. 0 on bad arguments. */
size_t pd_decompose_workspace_size(const pd_shape *shape, int32_t terms);

/* Theta~ by columns (CSC; equivalently the CSR of its transpose).
 *   shape   n1 x n2, channels = 1, levels >= 1 (as for pd_fwt).
 *   op      PD_OP_PC with FP64 taps [m][2R+1][2R+1] and mult [m][n2][n1] (device).
 *   eta     >= 0 (0: every nonzero of A_k kept, Theta~ = Theta up to rounding).
 *   capacity  room in rows / vals (device int32 / double); *nnz (host) gets the
 *           number of entries of Theta~; col_ptr (device int64 [n1 n2 + 1]) is always
 *           written; rows within a column ascend.  If nnz > capacity the entries are
 *           not all written and PD_ERR_WORKSPACE is returned (call again with
 *           capacity >= nnz; capacity 0 with rows = vals = NULL only counts).
 * The FP64 sums are accumulated with atomic adds in no fixed order: two calls agree
 * to rounding, and an entry that cancels can be exactly zero in one call and not
 * in the other, so a count from one call may be short for the next by a few
 * entries (size with some slack; col_ptr / rows / vals of one call are consistent).
 * Synchronises the host with `stream` (the thresholds are chosen on the host).
 * Errors: PD_ERR_ARG, PD_ERR_SHAPE, PD_ERR_TAU (eta), PD_ERR_WORKSPACE,
 * PD_ERR_UNSUPPORTED (not PD_OP_PC), PD_ERR_HIP. */
int pd_decompose(const pd_shape *shape, const pd_operator *op, const pd_wavelet *wav, double eta, int64_t capacity,
                 int64_t *nnz, int64_t *col_ptr, int32_t *rows, double *vals, void *workspace, size_t ws_bytes,
                 void *stream);

/* Diagnostics: per-launch kernel timing.  While enabled, every kernel launch
 * made by pd_solve / pd_solve_batched / pd_backward / pd_fwt / pd_wsolve /
 * pd_admm_solve (its iteration loop) / pd_decompose is bracketed by
 * two HIP events recorded on its launch stream, keyed by kernel class and
 * decomposition level.  Adds one event pair per launch; not thread-safe.   */
typedef enum {
    PD_K_BLUR = 1,      /* r = H x - f0, s = H^T r (one or two launches)        */
    PD_K_SYNTH = 2,     /* one synthesis level (level = decomposition level)   */
    PD_K_ANALYSIS = 3,  /* one analysis level with the fused prox              */
    PD_K_COARSE = 4,    /* all coarse levels of an iteration in one workgroup
                           per channel (or per image)                          */
    PD_K_OTHER = 5,     /* copies and set-up                                   */
    PD_K_WRES = 6,      /* wavelet domain: u = Theta_L y - z0                  */
    PD_K_WPROX = 7,     /* wavelet domain: Theta_L^T u, prox and momentum      */
    PD_K_FFT = 8,       /* ADMM-PC: one 2-D FFT pass over the m planes (level 0/1
                           forward rows/columns, 2/3 inverse rows/columns)     */
    PD_K_ADMM = 9,      /* ADMM-PC element-wise steps (level 1 spectral, 2 f and
                           multipliers, 3 zeta and z)                          */
    PD_K_DECOMP = 10,   /* Algorithm 1: level 0 probe convolutions, 1 multiplier,
                           2 spreading of B_k columns over A~_k, 3 count, 4 fill */
    PD_K_SYNTH2 = 11,   /* two synthesis levels in one launch (level = the finer) */
    PD_K_JPROX = 12,    /* joint colour prox over the whole coefficient plane  */
    PD_K_SYNTH3 = 13,   /* three synthesis levels in one launch (level = the
                           finest)                                             */
    PD_K_ANALYSIS2 = 14 /* two analysis levels with the fused prox in one
                           launch (level = the finer)                          */
} pd_kernel_class;

/* Start (enable != 0) or stop recording.  Starting clears the record. */
int pd_timing_enable(int32_t enable);

/* Waits for the recorded events and writes up to max_rows rows (kernel
 * class, level, launches, total milliseconds) to the host arrays; *rows gets
 * the number of rows available. */
int pd_timing_read(int32_t max_rows, int32_t *kclass, int32_t *level, int64_t *launches,
                   double *total_ms, int32_t *rows);

/* Graph replay of the iteration loop (default on).  pd_solve runs the
 * iterations between its first and last in chunks of 64 whose launches are
 * captured once into a HIP graph (on a library-owned stream, not the
 * caller's) and replayed on the caller's stream; the kernels then read the
 * iteration number from the workspace.  Results are bitwise the same with
 * and without it.  A chunk is captured when the call replays it at least 4
 * times (>= 258 iterations) and reused by later calls with the same
 * arguments (up to 32 cached; an evicted graph is destroyed once its last
 * launch has completed).  Off while timing is enabled and in pd_backward's
 * recomputation.  Process-wide; not thread-safe. */
int pd_graphs_enable(int32_t enable);

/* Fusion of the three (or, with two fine levels, two) coarsest fine synthesis
 * levels into one launch, and of the two coarsest fine analysis levels of an
 * iteration (one channel per tile set) into one launch (default on; results
 * are bitwise the same either way).  Process-wide; not thread-safe. */
int pd_fuse_enable(int32_t enable);

/* Short description of a pd_status code. */
const char *pd_strerror(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* PD_H */
