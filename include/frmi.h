/*
 * frmi.h -- C ABI of the MI355X (gfx950) implementation of fast-resolve's
 * interferometric response operator (Roth et al., arXiv 2406.09144).
 *
 * The operators follow the paper's statement of the problem:
 *   - R, the measurement equation of Sec. 2 (Eq. 1) with scalar gains G = 1:
 *       V_k = sum_ij I_ij a_ij exp(-2 pi i [u_k l_i + v_k m_j + w_k (n_ij - 1)]),
 *     l_i = (i - nx/2) dx, m_j = (j - ny/2) dy, n_ij = sqrt(1 - l_i^2 - m_j^2),
 *     a_ij = 1/n_ij with FR_DIVIDE_BY_N, else 1; (u, v, w) = uvw * nu / c.
 *   - R^+, its adjoint in the real inner product <p, q> = Re sum conj(p) q
 *     (the sky is real, Sec. 3.1.1), giving the dirty image R^+ N^-1 V (Sec. 3.2).
 *   - N^-1 = diag(weight) (Sec. 3.1.2).
 *   - R' = R^+ N^-1 R and its PSF-convolution approximation (Sec. 3.3.2), and the
 *     noise-kernel approximation of N'^-1 (Sec. 3.3.3).
 *
 * Conventions for every call:
 *   - Arrays are C-contiguous.  Complex numbers are interleaved (re, im).
 *   - Precision is a property of the plan (FR_FP64 -> double / complex128,
 *     otherwise float / complex64) and every float buffer of a call on that plan
 *     uses it.  uvw and frequencies are always double.
 *   - "device" pointers must point to memory on the plan's device; "host"
 *     pointers to ordinary host memory.
 *   - An image stack is [B][n_chan][nx][ny]; channels are independent (the
 *     operators are block-diagonal over channels).  Visibilities are
 *     [n_row][n_chan].
 *   - stream is a hipStream_t (NULL = the null stream).  Operator calls are
 *     asynchronous: they return after enqueueing; outputs are valid once the
 *     stream reaches that point.  Plan and PSF objects are read-only after
 *     creation and may be used from several streams at once.  Per-call scratch
 *     comes from an arena owned by the library for each (device, stream) pair:
 *     device memory that grows on demand (hipMalloc, outside the stream) and is
 *     reused by later calls on the same stream, which run in order; calls on
 *     different streams never share it.  fr_scratch_stats reports its use and
 *     fr_scratch_trim returns it to the device.
 *   - The caller owns every input/output buffer and the stream; the library
 *     owns ctx, plan and psf objects until the matching *_destroy.
 *   - Errors are returned as status codes (never exceptions, never abort);
 *     fr_last_error() gives a thread-local message for the last non-OK status.
 *     Invalid arguments return FR_EINVAL before anything is enqueued.
 *     Asynchronous device faults surface at a later call or synchronisation.
 */
#ifndef FRMI_H
#define FRMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_ctx fr_ctx;   /* one device */
typedef struct fr_plan fr_plan; /* uvw/frequencies bucketed on the grid, kernel parameters */
typedef struct fr_psf fr_psf;   /* response kernel K_R and noise kernel K_N per channel */
typedef struct fr_cf fr_cf;     /* correlated-field amplitude model on one grid */

enum fr_status {
    FR_OK = 0,
    FR_EINVAL = -1,       /* bad argument, shape or flag */
    FR_ENOMEM = -2,       /* device allocation failed */
    FR_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
    FR_EUNSUPPORTED = -4, /* valid request the library does not implement */
    FR_EBUSY = -5
};

enum fr_plan_flags {
    FR_FP64 = 1,        /* double precision buffers and arithmetic */
    FR_DIVIDE_BY_N = 2, /* include the 1/n factor of the w-term C(l, w) (Sec. 2) */
    FR_COPLANAR = 4,    /* treat every w as 0 (the paper's coplanar case, Sec. 3.3.2) */
    FR_W_TAYLOR = 8,    /* expand the w-term in a Taylor series when that needs fewer
                           planes than improved w-stacking at this epsilon */
    FR_VECTOR_SPREAD = 16 /* grid with the vector-unit spread even where the plan
                             would take the matrix-core one (FP32, W <= 8, runs of
                             4 or more records on average); same tiles, same bound */
};

enum fr_lik_mode { FR_LIK_EXACT = 0, FR_LIK_FAST = 1 };

/* kernel factor of fr_periodic_conv */
enum fr_conv_mode { FR_CONV_MUL = 0, FR_CONV_DIV = 1, FR_CONV_MUL_SQRT = 2, FR_CONV_DIV_SQRT = 3 };

enum fr_op {
    FR_OP_DEGRID = 0,
    FR_OP_GRID = 1,
    FR_OP_RNR_APPROX = 2,
    FR_OP_RNR_EXACT = 3,
    FR_OP_LIK_EXACT = 4,
    FR_OP_LIK_FAST = 5,
    FR_OP_CG = 6,
    FR_OP_MAKE_PSF = 7
};

/* Gridder parameters chosen by fr_plan_create (read-only). */
typedef struct fr_plan_info {
    int64_t nx, ny;         /* image */
    int64_t nu, nv;         /* oversampled uv grid */
    int64_t n_row, n_chan;
    int precision;          /* 32 or 64 */
    int support;            /* W: kernel width in uv cells */
    double beta;            /* ES kernel shape, phi(z) = exp(beta (sqrt(1 - z^2) - 1)) */
    int coplanar;           /* 1: single plane, no w kernel */
    int n_planes;           /* w-planes per channel */
    int w_support;          /* kernel width along w (planes) */
    double w_beta;
    double w0, dw;          /* plane p sits at w0 + p dw (wavelengths) */
    double eps_bound;       /* a-priori bound on the gridding error used to pick W */
    int tile;               /* uv tile side in cells */
    int64_t n_workitems;
    size_t resident_bytes;  /* device memory the plan holds */
    int w_taylor;           /* 1: the planes are Taylor terms in w, not w-planes */
    double records_per_run; /* sorted records per run of equal (bucket, base cell) */
    int matrix_spread;      /* 1: fr_grid spreads on the matrix cores (FP32, support <= 8,
                               >= 4 records per run); 0: on the vector units */
    int paired_degrid;      /* 1: fr_degrid interpolates two records of one base cell per
                               thread from the same tile reads (FP32, >= 4 records per run) */
    int64_t degrid_slots;   /* footprint interpolations fr_degrid issues: pair-list
                               entries when paired, else one per visibility */
    int64_t active_tiles;   /* uv tiles (tile x tile cells) whose planes can be non-zero,
                               summed over channels: fr_degrid reads and fr_grid writes
                               only these */
    int64_t active_tile_cols; /* tile columns holding an active tile, summed over
                               channels: the w-plane column and row transforms touch only
                               these columns */
} fr_plan_info;

/* Library version string. */
const char *fr_version(void);

/* Thread-local message of the last non-OK status (empty string if none). */
const char *fr_last_error(void);

/* Bind device `device` (hipSetDevice numbering).  Returns FR_EINVAL for a bad
 * index, FR_EHIP if the device cannot be used. */
int fr_ctx_create(int device, fr_ctx **out);
void fr_ctx_destroy(fr_ctx *ctx);

/*
 * Plan: bucket every (row, channel) visibility onto the oversampled grid.
 *   uvw_m    host [n_row][3] double, metres
 *   freq_hz  host [n_chan] double, Hz (> 0)
 *   nx, ny   image size, powers of two in [16, 8192]
 *   dx, dy   pixel sizes (radians, > 0); the field must satisfy l^2 + m^2 < 1
 *   epsilon  requested relative L2 accuracy of R and R^+ against the direct
 *            sums, in [1e-14, 1e-1]; FP32 plans accept epsilon >= 1e-6
 *   flags    FR_FP64 | FR_DIVIDE_BY_N | FR_COPLANAR | FR_W_TAYLOR | FR_VECTOR_SPREAD
 *            FR_W_TAYLOR: with t = (n - 1) - yc in [-h, h] over the image, write
 *            exp(-2 pi i w t) = sum_j (2 pi w h)^j / j! (-i t / h)^j and keep the
 *            J + 1 terms whose truncation, (2 pi w_max h)^(J+1) / (J+1)!, is below
 *            epsilon / 8: term j is a 2-D plane of the image times (-i t/h)^j,
 *            weighted per visibility by (2 pi w h)^j / j!.  Used only when
 *            2 pi w_max h <= 1 (no term above 1) and J + 1 is below the plane count
 *            of improved w-stacking (small w: short arrays, narrow fields);
 *            otherwise the plan stays w-stacked.
 *   n_wplanes 0 = derive from epsilon; otherwise the number of w-planes to use
 *            (must be >= the derived minimum)
 * The method itself is exact (Sec. 2); the gridder reaches it up to epsilon with
 * an exponential-of-semicircle kernel, 2x oversampling and improved w-stacking
 * (the kernel also runs along w).  Enqueues on the null stream and synchronises.
 * Errors: FR_EINVAL (shapes, ranges, flags), FR_ENOMEM, FR_EHIP.
 */
int fr_plan_create(fr_ctx *ctx, const double *uvw_m, int64_t n_row, const double *freq_hz,
                   int64_t n_chan, int64_t nx, int64_t ny, double dx, double dy, double epsilon,
                   int flags, int n_wplanes, fr_plan **out);
void fr_plan_destroy(fr_plan *plan);
int fr_plan_get_info(const fr_plan *plan, fr_plan_info *info);

/* Inspection of a plan's bucketing (for tests and tools; synchronous, host arrays,
 * any output may be NULL).  Visibility v = row * n_chan + chan has the 64-bit
 * sort key  bucket << 10 | (a * 32 + b),  bucket = (chan * n_first_planes +
 * first w-plane) * n_tiles + tile, (a, b) its base cell inside the 32 x 32 uv tile:
 *   keys          [n_vis]: the key of every visibility, in input order;
 *   perm          [n_vis]: perm[k] = v of the k-th record in the plan's order (a
 *                 stable sort of the keys);
 *   bucket_start  [n_keys + 1]: first record position of every bucket (and n_vis),
 *                 read back from the plan's degridding work items after checking
 *                 that they, and the gridding items, tile each bucket exactly;
 *   n_keys        number of buckets.
 * Errors: FR_EHIP if the work items are inconsistent. */
int fr_plan_export_order(const fr_plan *plan, uint64_t *keys, uint32_t *perm, int64_t *bucket_start,
                         int64_t *n_keys);

/* R (Sec. 2, Eq. 1): img device [n_chan][nx][ny] real -> vis device [n_row][n_chan]
 * complex.  Overwrites vis. */
int fr_degrid(fr_plan *plan, const void *img, void *vis, void *stream);

/* N^-1 R (Sec. 3.1.2 with Sec. 2): vis = weight * (R img), the weights applied as
 * the visibilities are stored.  The adjoint of fr_grid with the same weights in
 * the real inner product (the gradient of gridding with respect to its input
 * visibilities).  img device [n_chan][nx][ny] real, weight device [n_row][n_chan]
 * real (required), vis device [n_row][n_chan] complex, overwritten. */
int fr_degrid_weighted(fr_plan *plan, const void *img, const void *weight, void *vis, void *stream);

/* R^+ N^-1 (Sec. 3.2): vis device [n_row][n_chan] complex, weight device
 * [n_row][n_chan] real or NULL (= 1) -> img device [n_chan][nx][ny] real, the dirty
 * image when vis are the data.  Overwrites img. */
int fr_grid(fr_plan *plan, const void *vis, const void *weight, void *img, void *stream);

/*
 * Response and noise kernels (Sec. 3.3.2, Sec. 3.3.3), per channel:
 *   PSF0 = R0^+ N^-1 R0 delta on the doubled 2nx x 2ny grid (R0 = R with w := 0 and
 *          no 1/n), computed by gridding the weights; its offset -nx row and -ny
 *          column are set to zero so that it is periodically even;
 *   K_R  = Re rfft2(ifftshift(PSF0))                  -> [2nx][ny + 1]
 *   K_N  = eps + max(Re fft2(ifftshift(crop(PSF0))), 0) -> [nx][ny/2 + 1]
 *          where crop keeps offsets [-n/2, n/2): the closed-form minimiser of the
 *          noise-kernel fit of Sec. 3.3.3.
 *   weight   device [n_row][n_chan] real or NULL (= 1)
 *   eps_noise > 0: the regulariser eps of Sec. 3.3.1 (N' = R^+ N^-1 R + eps 1);
 *             < 0: -eps_noise times the PSF peak (sum of weights) of each channel.
 * The PSF object records the plan's 1/n factors (applied on both sides of the
 * convolution when the plan has FR_DIVIDE_BY_N).  Synchronises `stream`.
 */
int fr_make_psf_kernel(fr_plan *plan, const void *weight, double eps_noise, fr_psf **out,
                       void *stream);

/* Build a PSF object from caller-supplied kernels (e.g. precomputed elsewhere).
 *   K_R   device [n_chan][2nx][ny + 1] real (required)
 *   K_N   device [n_chan][nx][ny/2 + 1] real, entries > 0, or NULL (FAST
 *         likelihood then unavailable)
 *   nfac  device [nx][ny] real diagonal D applied on both sides, or NULL (= 1)
 *   flags FR_FP64 or 0 (precision of all three arrays)
 * Copies the arrays; synchronises `stream`. */
int fr_psf_create(fr_ctx *ctx, int64_t nx, int64_t ny, int64_t n_chan, const void *K_R,
                  const void *K_N, const void *nfac, int flags, fr_psf **out, void *stream);

/* Reduced PSF support (Sec. 3.3.2: neglecting the PSF sidelobes lets the zero
 * padding shrink, at the price of a less accurate R'): a new PSF object whose
 * response kernel keeps the PSF0 offsets |dx| <= hx, |dy| <= hy only, on a
 * px x py periodic grid with px the smallest even 2^p, 3 2^p or 5 2^p >= nx + hx
 * (py likewise), so that the cropped convolution stays linear:
 *   K_R' = Re rfft2(PSF0 truncated, offset d at index d mod p) -> [n_chan][px][py/2 + 1]
 * fr_apply_RNR_approx, the FAST likelihood and CG then convolve with the
 * truncated PSF on the smaller grid.  K_N and the 1/n factors are copied.
 *   psf     a PSF object with the full doubled-grid kernel (px = 2nx, py = 2ny),
 *           not modified; 0 <= hx < nx, 0 <= hy < ny.
 * The caller owns *out (fr_psf_destroy).  Synchronises `stream`. */
int fr_psf_reduce(const fr_psf *psf, int64_t hx, int64_t hy, fr_psf **out, void *stream);

/* Periodic grid px x py of the object's response kernel (2nx x 2ny unless reduced). */
int fr_psf_get_padding(const fr_psf *psf, int64_t *px, int64_t *py);

/* Copy the kernels out (either pointer may be NULL): K_R [n_chan][px][py/2 + 1],
 * K_N as above. */
int fr_psf_get_kernels(const fr_psf *psf, void *K_R, void *K_N, void *stream);
void fr_psf_destroy(fr_psf *psf);

/* R' x ~ D P^+ FFT^-1[K_R FFT[P D x]] (Sec. 3.3.2): zero-padded linear convolution
 * with the doubled-grid PSF (P pads to the object's px x py grid: 2nx x 2ny, or the
 * reduced grid of fr_psf_reduce).  x, y device [B][n_chan][nx][ny] real, y != x. */
int fr_apply_RNR_approx(fr_psf *psf, const void *x, void *y, int64_t B, void *stream);

/* Fixed device workspace of fr_apply_RNR_approx_noalloc, per GPU (bytes). */
#define FR_NOALLOC_SCRATCH_BYTES (64u << 20)

/* fr_apply_RNR_approx for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operator, arguments and kernels, but the half-spectrum workspace is a
 * fixed array of FR_NOALLOC_SCRATCH_BYTES in the library's device image, one per
 * GPU, held until the process ends; the call performs no device allocation or
 * release.  It needs B * n_chan * nx * (py/2) complex elements (py = 2ny, or the
 * reduced grid) of the PSF's precision, at most FR_NOALLOC_SCRATCH_BYTES
 * (e.g. FP32 512^2 with B * n_chan <= 32, 1024^2 with <= 8); larger requests
 * return FR_EINVAL before anything is enqueued.  A context must have been created
 * on the PSF's device (fr_ctx_create finds the workspace's device address there).
 * Every such call on one GPU uses the same workspace, so calls that overlap on a
 * GPU (different streams, or host threads without ordering) race on it: the
 * caller orders them, e.g. by issuing them on one stream. */
int fr_apply_RNR_approx_noalloc(fr_psf *psf, const void *x, void *y, int64_t B, void *stream);

/* R' x = R^+ N^-1 R x evaluated exactly (major cycle, Sec. 3.3.4).
 * weight device [n_row][n_chan] or NULL; x, y device [B][n_chan][nx][ny]. */
int fr_apply_RNR_exact(fr_plan *plan, const void *weight, const void *x, void *y, int64_t B,
                       void *stream);

/*
 * Likelihood Hamiltonian and its gradient with respect to the log-sky s, with
 * I = exp(s) + i_fixed, for a batch of B samples; the constant 1/2 ln|2 pi N|
 * is dropped.
 *   FR_LIK_EXACT (eq. ham, Sec. 3.1.2): data = visibilities [n_row][n_chan];
 *       H = 1/2 sum w |V - R I|^2,  g = exp(s) * R^+ [w (R I - V)]   (plan required)
 *   FR_LIK_FAST (eq. ham_new, Sec. 3.3.1 with Sec. 3.3.2-3.3.3): data = dirty
 *       image d [n_chan][nx][ny]; r = d - R' I, q = N'^-1 r,
 *       H = 1/2 <r, q>,  g = -exp(s) * R' q                        (psf required)
 *   s, grad  device [B][n_chan][nx][ny];  i_fixed device [n_chan][nx][ny] or NULL
 *   weight   device [n_row][n_chan] or NULL (EXACT only)
 *   inv_power device [nx][ny/2 + 1] real 1/P(k) (r2c half of an even spectrum) or
 *            NULL; adds the prior term 1/2 s^T S^-1 s (S^-1 = F^-1 diag(1/P) F per
 *            channel) to H and S^-1 s to g
 *   H        device [B] double (accumulated in double)
 */
int fr_likelihood_grad(fr_plan *plan, fr_psf *psf, int mode, const void *s, const void *i_fixed,
                       const void *data, const void *weight, const void *inv_power, int64_t B,
                       void *grad, double *H, void *stream);

/*
 * Conjugate gradients (Hestenes-Stiefel, x0 = 0, no preconditioner) on
 *   A x = D_s R' D_s x + S^-1 x = b
 * with R' the PSF convolution of `psf` (or, if psf is NULL, the exact R^+ N^-1 R
 * of `plan` with `weight`), D_s = diag(diag) (NULL = identity) and
 * S^-1 = F^-1 diag(inv_power) F (NULL = no prior term).  The metric solve MGVI
 * uses in the minor cycle (Sec. 3.3.5).
 *   b, x        device [n_chan][nx][ny] (one system over all channels)
 *   inv_power   device [nx][ny/2 + 1] or NULL
 *   diag        device [n_chan][nx][ny] or NULL
 *   maxiter     >= 0; rtol >= 0 stops once ||r_k|| <= rtol ||b||
 *   resid_hist  device [maxiter + 1] double: ||r_k||, entries after the last
 *               iteration are left untouched
 *   iters_done  device int: iterations performed
 * Inner products and the alpha/beta recurrences are double precision on the
 * device; no host synchronisation inside the loop.
 */
int fr_cg_solve(fr_plan *plan, fr_psf *psf, const void *weight, const void *inv_power,
                const void *diag, const void *b, void *x, int maxiter, double rtol,
                double *resid_hist, int *iters_done, void *stream);

/*
 * Periodic convolution with a real even kernel given by its r2c half spectrum on
 * the nx x ny grid (noise kernel of Sec. 3.3.3, Gaussian-process prior):
 *   y = F^-1 diag(f(K)) F x,  f = K, 1/K, sqrt K or 1/sqrt K for mode
 *   FR_CONV_MUL, FR_CONV_DIV, FR_CONV_MUL_SQRT, FR_CONV_DIV_SQRT.
 * With K = P(k) and FR_CONV_MUL_SQRT this maps standardised excitations xi to the
 * log-sky s = A xi of covariance S (the exponentiated Gaussian process of the
 * diffuse prior, Sec. 3.1.1); FR_CONV_DIV_SQRT is A^-1.
 *   K      device [nk][nx][ny/2 + 1] real (> 0 for the DIV and SQRT modes);
 *          image g uses K[g % nk]
 *   x, y   device [n_img][nx][ny] real, y != x; fp64 selects double.
 * nx, ny powers of two in [4, 8192]. */
int fr_periodic_conv(fr_ctx *ctx, const void *K, int64_t nk, int mode, const void *x, void *y,
                     int64_t n_img, int64_t nx, int64_t ny, int fp64, void *stream);

/*
 * MGVI pieces for the minor cycle (Sec. 3.3.5) in standardised coordinates: the
 * log-sky is s = A xi (A as fr_periodic_conv with power P, FR_CONV_MUL_SQRT) and
 * the FAST likelihood (eq. ham_new) has the Fisher metric
 *   M = 1 + A D R' N'^-1 R' D A,   D = diag(diag) = diag(exp s) at the expansion point,
 * with R' the PSF convolution of `psf` (any padding) and N'^-1 its noise kernel.
 *   power  device [nx][ny/2 + 1] real P(k) > 0 (shared by the channels)
 *   diag   device [n_chan][nx][ny] or NULL (= 1)
 *   vectors device [n_chan][nx][ny]: one system over all channels.
 * fr_mgvi_metric_apply: y = M x (y != x).
 * fr_mgvi_draw: xi = eta0 + A D R' N'^-1/2 eta1, which has covariance M for white
 *   eta0, eta1 (the random numbers come from the caller); xi aliases neither.
 * fr_mgvi_solve: M x = b by conjugate gradients (Hestenes-Stiefel, x0 = 0, FP64
 *   scalars on the device, no host synchronisation; arguments as fr_cg_solve).
 *   With b from fr_mgvi_draw, x ~ N(0, M^-1) is an MGVI sample offset; with b a
 *   gradient, x is the natural-gradient step.
 * The PSF object must carry a noise kernel. */
int fr_mgvi_metric_apply(fr_psf *psf, const void *power, const void *diag, const void *x, void *y,
                         void *stream);
int fr_mgvi_draw(fr_psf *psf, const void *power, const void *diag, const void *eta0,
                 const void *eta1, void *xi, void *stream);
int fr_mgvi_solve(fr_psf *psf, const void *power, const void *diag, const void *b, void *x,
                  int maxiter, double rtol, double *resid_hist, int *iters_done, void *stream);

/*
 * Correlated-field amplitude model of the diffuse-emission prior (the power
 * spectrum of the exponentiated Gaussian process of Sec. 3.1.1, inferred with
 * the hyperparameters listed in the prior-parameter appendices).  Reading of the
 * model, whose definition the paper defers to earlier work:
 *   - zero-mode std, fluctuations, flexibility and asperity are lognormal with
 *     the given mean and standard deviation (exp(mu + sigma xi), sigma^2 =
 *     ln(1 + std^2/mean^2), mu = ln mean - sigma^2/2; a mean of 0 gives 0);
 *     the average log-log slope is normal (mean + std xi);
 *   - over the J distinct non-zero |k| of the grid (integer frequency units), at
 *     t = ln|k| ascending with steps d_j (d_0 = 0): the local slope
 *     v_j = flex sum_{i<=j} sqrt(d_i) xi_v_i (a Wiener process), its integral with
 *     a rougher part y_j = sum_{i<=j} [(v_i-1 + v_i) d_i / 2 + flex asp sqrt(d_i) xi_y_i],
 *     and the log-amplitude logA_j = slope (t_j - t_0) + y_j - y_J (t_j - t_0)/(t_J - t_0);
 *   - P = fluct^2 nx ny A^2 / sum_j mult_j A_j^2 at k != 0 (mult_j: frequencies
 *     of the full grid in bin j), P(0) = zm^2 nx ny: the field without its zero
 *     mode has variance fluct^2;
 *   - log-sky s = offset + F^-1 sqrt(P) F xi_field.
 * fr_cf_create: bins of an nx x ny grid (powers of two in [4, 8192]); synchronous.
 * fr_cf_power:
 *   prior     host double [11]: zero-mode offset, zero-mode std mean, std;
 *             fluctuations mean, std; slope mean, std; flexibility mean, std;
 *             asperity mean, std
 *   xi_hyper  device double [5] standardised excitations (zero-mode std,
 *             fluctuations, slope, flexibility, asperity)
 *   xi_v, xi_y device double [J] (fr_cf_num_bins)
 *   power     device [nx][ny/2 + 1] real (r2c half spectrum; fp64 selects double),
 *             usable as the power of fr_periodic_conv and of the MGVI calls.
 * fr_cf_logsky: s = offset + F^-1 sqrt(P) F xi for n_img images; power as
 *   written by fr_cf_power, xi and s device [n_img][nx][ny] real, s != xi.
 */
int fr_cf_create(fr_ctx *ctx, int64_t nx, int64_t ny, fr_cf **out);
int fr_cf_num_bins(const fr_cf *cf, int64_t *n_bins);
int fr_cf_power(fr_cf *cf, const double *prior, const double *xi_hyper, const double *xi_v,
                const double *xi_y, void *power, int fp64, void *stream);
int fr_cf_logsky(fr_cf *cf, const void *power, double offset, const void *xi, void *s, int64_t n_img,
                 int fp64, void *stream);
void fr_cf_destroy(fr_cf *cf);

/* Device bytes a call of `op` with batch B needs beyond its inputs and outputs,
 * plus the resident plan/psf bytes.  Host-only, no GPU work.  scratch_bytes bounds
 * the per-call scratch the call takes from its stream's arena (regions rounded to
 * 256 bytes, prior-term scratch included for the ops that take one); for
 * FR_OP_MAKE_PSF it adds a bound on the doubled-field plan the call builds and
 * frees.  Admission control can sum it over calls in flight. */
int fr_query_footprint(const fr_plan *plan, const fr_psf *psf, int op, int64_t B,
                       size_t *scratch_bytes, size_t *resident_bytes);

/* Scratch arena of (ctx's device, stream): `held` = device bytes it owns,
 * `peak_in_use` = the largest sum of regions live at once since the last reset
 * (reset != 0 restarts the count after reading).  Host-only. */
int fr_scratch_stats(fr_ctx *ctx, void *stream, int reset, size_t *peak_in_use, size_t *held);

/* Synchronise `stream`, then free the device memory of its arena (the next call on
 * the stream allocates again).  FR_EBUSY if a call is using it. */
int fr_scratch_trim(fr_ctx *ctx, void *stream);

/* Failure injection for tests of the error paths: after `after` more successful
 * device allocations by the library, the next one fails as out of memory (the
 * call returns FR_ENOMEM and releases what it had taken).  One failure per
 * injection; -1 cancels a pending one. */
int fr_inject_alloc_failure(int64_t after);

/* Per-kernel timing for measurement (off by default, process-wide).  While
 * enabled, each instrumented kernel launch is bracketed by two hipEvents
 * recorded on the launch's own stream.  fr_profile_query synchronises the
 * recorded events of kernel `name` and returns the number of launches and their
 * summed duration in milliseconds (0 launches for an unknown name).  Names:
 * "degrid", "grid", "grid_assemble", "zero", "wplane_rows_fwd", "wplane_cols_fwd",
 * "wplane_cols_inv", "wplane_rows_inv", "psfconv_rows_r2c", "psfconv_cols",
 * "psfconv_rows_c2r", "pconv_rows_r2c", "pconv_cols", "pconv_rows_c2r".
 * fr_profile_reset drops every record. */
int fr_profile_enable(int on);
int fr_profile_reset(void);
int fr_profile_query(const char *name, int64_t *launches, double *total_ms);

/* Building block exposed for testing: in-place 2D complex FFT of a device array
 * [batch][n0][n1] (n0, n1 of the form 2^p, 3 2^p or 5 2^p, 2 <= n <= 16384, FP64 up
 * to 8192),
 * sign -1 forward, +1 inverse, unnormalised.  fp64 selects complex128. */
int fr_fft2(fr_ctx *ctx, void *data, int64_t batch, int64_t n0, int64_t n1, int sign, int fp64,
            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FRMI_H */
