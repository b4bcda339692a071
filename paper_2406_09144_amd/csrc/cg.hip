// Conjugate gradients on A x = D_s R' D_s x + S^-1 x = b and on the MGVI metric:
// the solves MGVI uses to apply the inverse metric in the minor cycle (Sec. 3.3.5).
// Hestenes-Stiefel recurrences with x0 = 0 and no preconditioner.
//
// Vectors are in the plan/PSF precision; <r, r>, <p, A p>, alpha and beta are
// double precision scalars that live on the device.  Every kernel reads them
// from device memory, so the host enqueues `maxiter` iterations without ever
// synchronising; once ||r|| <= rtol ||b|| a device flag turns the remaining
// kernels into no-ops.  Reductions need no fences or atomics: a kernel writes
// per-block partial sums and every block of the next kernel adds them itself,
// in the same fixed order, so all blocks agree on alpha and beta.
#include "conv.h"
#include "elementwise.h"
#include "objects.h"
#include "profiler.h"

namespace frmi {

struct CGState {
    double stop;  // rtol ||b||
    int done;
    int iters;
    // fused PSF-form loop: flag[k & 1] != 0 once iteration k (or an earlier one)
    // met the stopping test; flag[1] also carries the start test for k = 0
    int flag[2];
};

template <typename T> struct CGInit {
    const T *b;
    T *x, *r, *p;
    __device__ void operator()(int64_t i) const {
        const T v = b[i];
        x[i] = T(0);
        r[i] = v;
        p[i] = v;
    }
};

// rr[0] = <b, b> from the partials of k_dot_partials, stopping threshold, history
__global__ __launch_bounds__(kRedThreads) void k_cg_start(CGState *st, const double *rr_partials, int nparts,
                                                          double rtol, int maxiter, double *rr, double *hist) {
    const double s = block_sum_partials(rr_partials, nparts);
    if (threadIdx.x != 0) return;
    rr[0] = s;
    st->stop = rtol * sqrt(s);
    st->iters = 0;
    st->done = (s == 0.0 || maxiter == 0) ? 1 : 0;
    st->flag[0] = 0;
    st->flag[1] = st->done;
    hist[0] = sqrt(s);
}

// y = diag * x (or copy)
template <typename T> struct DiagMul {
    const T *d, *x;
    T *y;
    __device__ void operator()(int64_t i) const { y[i] = d ? d[i] * x[i] : x[i]; }
};

// Ap = diag * u + prior
template <typename T> struct DiagMulAdd {
    const T *d, *u, *prior;
    T *y;
    __device__ void operator()(int64_t i) const {
        T v = d ? d[i] * u[i] : u[i];
        if (prior) v += prior[i];
        y[i] = v;
    }
};

__device__ __forceinline__ bool cg_done(const CGState *st) {
    return __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// partials of <p, A p>
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_dot_pAp(const CGState *__restrict__ st, const T *__restrict__ p,
                                                            const T *__restrict__ Ap, int64_t n,
                                                            double *__restrict__ pAp_partials) {
    if (cg_done(st)) return;
    double s = grid_stride_sum(n, [&](int64_t i) { return (double)p[i] * (double)Ap[i]; });
    s = block_sum(s);
    if (threadIdx.x == 0) pAp_partials[blockIdx.x] = s;
}

// alpha = <r_k, r_k> / <p, A p>; x += alpha p, r -= alpha A p; partials of <r, r>.
// <r_k, r_k> lives in rr[k & 1] (two slots: iteration k reads one, writes the other)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_step(const CGState *__restrict__ st, T *__restrict__ x,
                                                         T *__restrict__ r, const T *__restrict__ p,
                                                         const T *__restrict__ Ap, int64_t n,
                                                         const double *__restrict__ pAp_partials, int n_pAp,
                                                         const double *__restrict__ rr, int k,
                                                         double *__restrict__ rr_partials) {
    if (cg_done(st)) return;
    __shared__ double alpha_sh;
    const double pAp = block_sum_partials(pAp_partials, n_pAp);
    if (threadIdx.x == 0) alpha_sh = rr[k & 1] / pAp;
    __syncthreads();
    const T a = (T)alpha_sh;
    double s = grid_stride_sum(n, [&](int64_t i) {
        const T pv = p[i], apv = Ap[i], xv = x[i], rv0 = r[i];
        x[i] = xv + a * pv;
        const T rv = rv0 - a * apv;
        r[i] = rv;
        return (double)rv * (double)rv;
    });
    s = block_sum(s);
    if (threadIdx.x == 0) rr_partials[blockIdx.x] = s;
}

// <r_k+1, r_k+1> -> rr[(k + 1) & 1], beta = its ratio to rr[k & 1], p = r + beta p; block 0 records the
// history and the stopping flag (blocks that already see the flag skip the
// update of p, which is no longer used)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_update_p(CGState *__restrict__ st, T *__restrict__ p,
                                                             const T *__restrict__ r, int64_t n,
                                                             const double *__restrict__ rr_partials, int n_rr,
                                                             double *__restrict__ rr, int k,
                                                             double *__restrict__ hist) {
    if (cg_done(st)) return;
    __shared__ double beta_sh;
    const double rn = block_sum_partials(rr_partials, n_rr);
    if (threadIdx.x == 0) {
        beta_sh = rn / rr[k & 1];
        if (blockIdx.x == 0) {
            rr[(k + 1) & 1] = rn;
            hist[k + 1] = sqrt(rn);
            st->iters = k + 1;
            if (sqrt(rn) <= st->stop) __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    const T beta = (T)beta_sh;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
        p[i] = r[i] + beta * p[i];
}

__global__ void k_cg_report(const CGState *st, int *iters_done) {
    if (threadIdx.x == 0) *iters_done = st->iters;
}

// ------------------------------------------------------------------ fused PSF-form iteration
// For A = D_s R'_PSF D_s + S^-1 with the full doubled-grid PSF, one iteration is
// three launches instead of nine:
//   1. row transforms of two images per channel on the doubled grid, a D_s p_k
//      and p_k, whose prologue first completes the previous step: with
//      alpha = <r, r> / <p, A p> of iteration k - 1,
//        x += alpha p_k-1,  r_k = r_k-1 - alpha A p_k-1,
//        <r_k, r_k> = <r, r> - 2 alpha <r, A p> + alpha^2 <A p, A p>,
//        beta = <r_k, r_k> / <r, r>,  p_k = r_k + beta p_k-1
//      (each workgroup forms the scalars from the partial sums of pass 3 of
//      iteration k - 1; workgroup 0 records the residual history and the stop
//      test);
//   2. column transforms, the first image multiplied by K_R, the second by the
//      prior embedded in the doubled grid (below);
//   3. inverse row transforms of both images of a row in one workgroup:
//      A p = D_s a y_R + y_S, and the partial sums of <p, A p>, <r, A p>,
//      <A p, A p> and <r, r> (r = r_k).
// A final launch applies the last step to x.  The scalars are those of the
// Hestenes-Stiefel recurrences (alpha and beta from the residual norms); only
// <r_k, r_k> is formed from the expansion of |r_k-1 - alpha A p_k-1|^2 with
// the dot products of the vectors themselves (as in the single-reduction CG of
// Chronopoulos and Gear), so that no separate pass over r_k is needed before
// beta.  The next iteration's pass 3 sums <r_k, r_k> from r_k directly.
// The prior S^-1 = F^-1 diag(1/P) F on the nx x ny periodic grid embeds in the
// doubled grid: the 2n-point transform of the zero-padded p at even frequencies
// 2k is the n-point transform of p at k, and a spectrum living on the even
// frequencies only transforms back to the n-periodic signal repeated, scaled by
// 1/4 (one 1/2 per axis).  So with H[2k1][2k2] = 4 / P(k1, k2) and H = 0 at every
// other frequency, the cropped linear convolution of the padded p with H is
// S^-1 p exactly (the same operator, in the same pipeline as R').

// H [2nx][ny + 1] from 1/P [nx][ny/2 + 1] (r2c halves)
template <typename T> struct PriorEmbed {
    const T *ip;
    T *H;
    int nx, ny;
    __device__ void operator()(int64_t i) const {
        const int w = ny + 1;
        const int f1 = (int)(i / w), f2 = (int)(i - (int64_t)f1 * w);
        H[i] = ((f1 | f2) & 1) ? T(0) : T(4) * ip[(int64_t)(f1 >> 1) * (ny / 2 + 1) + (f2 >> 1)];
    }
};

template <typename T> struct CGInitXR {
    const T *b;
    T *x, *r;
    __device__ void operator()(int64_t i) const {
        x[i] = T(0);
        r[i] = b[i];
    }
};

// The four FP64 sums of pass 3 over its n blocks (partials [block][4]), fixed
// order, returned to every thread of the workgroup
__device__ __forceinline__ void block_sum4_partials_all(const double *partials, int n, double out[4]) {
    __shared__ double sh[4][16];
    double v[4] = {0, 0, 0, 0};
    for (int k = threadIdx.x; k < n; k += blockDim.x)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            v[j] += __hip_atomic_load(partials + 4 * (int64_t)k + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_down(v[j], o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < 4; ++j) sh[j][wid] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[j][k];
        out[j] = t;
    }
    __syncthreads();
}

// Scalars of the step from iteration k - 1 to k: alpha, <r_k, r_k> and beta from
// <p, A p>, <r, A p>, <A p, A p>, <r, r> of iteration k - 1
struct CGStepScalars {
    double alpha, rn, beta;
};
__device__ __forceinline__ CGStepScalars cg_step_scalars(const double s[4]) {
    CGStepScalars c;
    c.alpha = s[3] / s[0];
    c.rn = fmax(s[3] - 2.0 * c.alpha * s[1] + c.alpha * c.alpha * s[2], 0.0);
    c.beta = c.rn / s[3];
    return c;
}

// Pass-1 prologue of iteration k.  Rows [0, n0) are the first image set (a D_s p),
// rows [n0, 2 n0) the second (p).  Workgroups skip the pass once an earlier
// iteration met the stopping test (and pass the flag on).  For k > 0 the first
// image set completes the previous step (x, r_k and p_k written); the second
// recomputes p_k from the same inputs without writing.
template <typename T> struct CGRowPro {
    T *x;
    const T *r_prev;  // r_k-1 (r_0 = b when k = 0)
    T *r_cur;         // r_k (k > 0)
    const T *p_prev, *Ap;
    T *p_cur;
    const T *d, *a;
    int nx, ny;
    int64_t n0;
    CGState *st;
    const double *parts;  // pass-3 partials of iteration k - 1, [n_parts][4]
    int n_parts;
    double *hist;
    int k;
    T alpha, beta;
    __device__ bool begin() {
        if (__hip_atomic_load(&st->flag[(k + 1) & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            if (threadIdx.x == 0) __hip_atomic_store(&st->flag[k & 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        alpha = beta = T(0);
        if (k == 0) return true;
        double s[4];
        block_sum4_partials_all(parts, n_parts, s);
        const CGStepScalars c = cg_step_scalars(s);
        alpha = (T)c.alpha;
        beta = (T)c.beta;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            hist[k] = sqrt(c.rn);
            st->iters = k;
            if (sqrt(c.rn) <= st->stop)
                __hip_atomic_store(&st->flag[k & 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        return true;
    }
    __device__ T operator()(int64_t row, int col) const {
        const bool second = row >= n0;
        const int64_t prow = second ? row - n0 : row;
        const int64_t q = prow * ny + col;
        T pv;
        if (k == 0) {
            pv = r_prev[q];
        } else {
            const T po = p_prev[q];
            const T rv = r_prev[q] - alpha * Ap[q];
            pv = rv + beta * po;
            if (!second) {
                x[q] += alpha * po;
                r_cur[q] = rv;
            }
        }
        if (second) return pv;
        p_cur[q] = pv;
        T v = pv;
        if (d) v *= d[q];
        if (a) v *= a[((int)prow & (nx - 1)) * ny + col];
        return v;
    }
};

// Pass-3 epilogue: A p = D_s a y_R + y_S; returns the pixel pair's shares of
// <p, A p>, <r, A p>, <A p, A p> and <r, r>
template <typename T> struct CGPairEpi {
    T *Ap;
    const T *p, *r, *d, *a;
    int nx, ny;
    __device__ SumN<4> operator()(int64_t row, int col, T y0, T y1, T s0, T s1) const {
        const int64_t q = row * ny + col;
        if (d) {
            y0 *= d[q];
            y1 *= d[q + 1];
        }
        if (a) {
            const T *pa = a + ((int)row & (nx - 1)) * ny + col;
            y0 *= pa[0];
            y1 *= pa[1];
        }
        y0 += s0;
        y1 += s1;
        Ap[q] = y0;
        Ap[q + 1] = y1;
        const double p0 = p[q], p1 = p[q + 1], r0 = r[q], r1 = r[q + 1];
        return SumN<4>{{p0 * y0 + p1 * y1, r0 * y0 + r1 * y1, (double)y0 * y0 + (double)y1 * y1,
                        r0 * r0 + r1 * r1}};
    }
};

// The last step: x += alpha p_K-1 and <r_K, r_K> into the history, unless an
// earlier iteration stopped; the iteration count.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_finish_fused(CGState *st, T *__restrict__ x,
                                                                 const T *__restrict__ p, int64_t n,
                                                                 const double *parts, int n_parts, int K,
                                                                 double *hist, int *iters_done) {
    const bool skip = K == 0 ||
                      __hip_atomic_load(&st->flag[(K + 1) & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    if (!skip) {
        double s[4];
        block_sum4_partials_all(parts, n_parts, s);
        const CGStepScalars c = cg_step_scalars(s);
        const T alpha = (T)c.alpha;
        for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
            x[i] += alpha * p[i];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            hist[K] = sqrt(c.rn);
            st->iters = K;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *iters_done = st->iters;
}

// The fused form applies to the full doubled-grid PSF (the prior embedding needs
// the 2n grid) with rows that fit the paired inverse pass.
static bool cg_fused_applies(const fr_psf *psf, bool prior) {
    return psf && psf->px == 2 * psf->nx && psf->py == 2 * psf->ny && (prior ? 2 : 1) * psf->ny <= 8192;
}

static size_t cg_fused_scratch(const fr_psf *psf, bool prior) {
    const size_t rs = psf->fp64 ? 8 : 4;
    const int64_t nx = psf->nx, ny = psf->ny, nc = psf->n_chan, n = nc * nx * ny;
    const int npart = prior ? 2 : 1;
    const int64_t nb3 = irfft_pair_blocks((int)ny, nc * nx, npart, 256, nullptr, nullptr);
    const size_t vec = scratch_round((size_t)n * rs);
    // partials: the pass-3 block count depends on the device's CU count; bound it by one block per row
    const size_t parts = scratch_round((size_t)(red_blocks(n) + 4 * std::max<int64_t>(nb3, nc * nx)) * 8);
    return scratch_round(sizeof(CGState)) + parts + scratch_round(2 * sizeof(double)) + 5 * vec +
           scratch_round((size_t)npart * nc * nx * ny * 2 * rs) + (prior ? scratch_round((size_t)2 * nx * (ny + 1) * rs) : 0);
}

template <typename T>
static void cg_solve_psf_fused(const fr_psf *psf, const T *inv_power, const T *diag, const T *b, T *x, int maxiter,
                               double rtol, double *hist, int *iters_done, hipStream_t st) {
    const int64_t nx = psf->nx, ny = psf->ny, nc = psf->n_chan, n = nc * nx * ny;
    const Ctx &ctx = *psf->ctx;
    const int npart = inv_power ? 2 : 1;
    const int M = (int)ny;  // packed width of the doubled rows
    const int log2M = ilog2(M);
    const int nb = red_blocks(n);
    const int64_t nb3 = irfft_pair_blocks(M, nc * nx, npart, ctx.n_cu, nullptr, nullptr);
    Scratch state(sizeof(CGState), st);
    Scratch partials((size_t)(nb + 4 * std::max<int64_t>(nb3, nc * nx)) * sizeof(double), st);
    double *rr_part = partials.as<double>(), *part3 = partials.as<double>() + nb;
    Scratch rr(2 * sizeof(double), st);
    Scratch rA(n * sizeof(T), st), rB(n * sizeof(T), st), pA(n * sizeof(T), st), pB(n * sizeof(T), st),
        Ap(n * sizeof(T), st);
    Scratch Y((size_t)npart * nc * nx * M * sizeof(c2<T>), st);
    Scratch H;
    if (inv_power) {
        H = Scratch((size_t)2 * nx * (ny + 1) * sizeof(T), st);
        map_async(PriorEmbed<T>{inv_power, H.as<T>(), (int)nx, (int)ny}, 2 * nx * (ny + 1), st);
    }
    CGState *S = state.as<CGState>();
    T *rbuf[2] = {rA.as<T>(), rB.as<T>()}, *pbuf[2] = {pA.as<T>(), pB.as<T>()};
    map_async(CGInitXR<T>{b, x, rbuf[0]}, n, st);
    k_dot_partials<T><<<dim3((unsigned)nb, 1), kRedThreads, 0, st>>>(rbuf[0], nullptr, n, rr_part);
    LAUNCH_CHECK();
    k_cg_start<<<1, kRedThreads, 0, st>>>(S, rr_part, nb, rtol, maxiter, rr.as<double>(), hist);
    LAUNCH_CHECK();
    ConvGeom g;
    g.n_img = npart * nc;
    g.rows_in = (int)nx;
    g.rows_out = (int)nx;
    g.n_in_cols = (int)ny;
    g.n_out_cols = (int)ny;
    g.log2M = log2M;
    g.log2Lc = ilog2(2 * nx);
    const T scale = T(1) / (T(2 * nx) * T(M));
    const T *a = psf->nfac.as<T>();
    for (int k = 0; k < maxiter; ++k) {
        // r_k in rbuf[k & 1], p_k in pbuf[k & 1]
        T *r_cur = rbuf[k & 1], *p_cur = pbuf[k & 1];
        const T *r_prev = rbuf[(k + 1) & 1], *p_prev = pbuf[(k + 1) & 1];
        CGRowPro<T> pro{x, k == 0 ? r_cur : r_prev, r_cur, p_prev, Ap.as<T>(), p_cur, diag, a, (int)nx, (int)ny,
                        nc * nx, S, part3, (int)nb3, hist, k, T(0), T(0)};
        {
            ProfScope prof("cg_rows_r2c", st);
            launch_rfft_rows<T>(ctx, g, pro, Y.as<c2<T>>(), st);
        }
        {
            ProfScope prof("cg_cols", st);
            launch_conv_cols<T>(ctx, g, Y.as<c2<T>>(), psf->KR.as<T>(), (int)nc, 0, scale, st, H.as<T>(),
                                inv_power ? nc : INT64_MAX, &S->flag[k & 1]);
        }
        {
            ProfScope prof("cg_rows_c2r", st);
            launch_irfft_rows_pair<T>(ctx, log2M, nc * nx, nc * nx, npart, (int)ny,
                                      CGPairEpi<T>{Ap.as<T>(), p_cur, r_cur, diag, a, (int)nx, (int)ny},
                                      Y.as<c2<T>>(), part3, &S->flag[k & 1], st);
        }
    }
    k_cg_finish_fused<T><<<dim3((unsigned)nb), kRedThreads, 0, st>>>(S, x, pbuf[(maxiter + 1) & 1], n, part3,
                                                                      (int)nb3, maxiter, hist, iters_done);
    LAUNCH_CHECK();
}

// The Hestenes-Stiefel loop around an operator apply(p, Ap) on n values.
template <typename T, class Apply>
void cg_run(int64_t n, const T *b, T *x, int maxiter, double rtol, double *hist, int *iters_done, hipStream_t st,
            Apply apply) {
    Scratch state(sizeof(CGState), st);
    const int nb = red_blocks(n);
    Scratch partials((size_t)2 * nb * sizeof(double), st);
    Scratch rr(2 * sizeof(double), st);
    double *pAp_part = partials.as<double>(), *rr_part = partials.as<double>() + nb;
    Scratch r(n * sizeof(T), st), p(n * sizeof(T), st), Ap(n * sizeof(T), st);
    CGState *S = state.as<CGState>();
    map_async(CGInit<T>{b, x, r.as<T>(), p.as<T>()}, n, st);
    k_dot_partials<T><<<dim3((unsigned)nb, 1), kRedThreads, 0, st>>>(r.as<T>(), nullptr, n, rr_part);
    LAUNCH_CHECK();
    k_cg_start<<<1, kRedThreads, 0, st>>>(S, rr_part, nb, rtol, maxiter, rr.as<double>(), hist);
    LAUNCH_CHECK();
    for (int k = 0; k < maxiter; ++k) {
        apply(p.as<T>(), Ap.as<T>());
        k_cg_dot_pAp<T><<<dim3((unsigned)nb), kRedThreads, 0, st>>>(S, p.as<T>(), Ap.as<T>(), n, pAp_part);
        LAUNCH_CHECK();
        k_cg_step<T><<<dim3((unsigned)nb), kRedThreads, 0, st>>>(S, x, r.as<T>(), p.as<T>(), Ap.as<T>(), n, pAp_part,
                                                                  nb, rr.as<double>(), k, rr_part);
        LAUNCH_CHECK();
        k_cg_update_p<T><<<dim3((unsigned)nb), kRedThreads, 0, st>>>(S, p.as<T>(), r.as<T>(), n, rr_part, nb,
                                                                      rr.as<double>(), k, hist);
        LAUNCH_CHECK();
    }
    k_cg_report<<<1, 64, 0, st>>>(S, iters_done);
    LAUNCH_CHECK();
}

size_t cg_scratch(const fr_plan *pl, const fr_psf *psf, bool prior) {
    if (cg_fused_applies(psf, prior)) return std::max(cg_fused_scratch(psf, prior), cg_fused_scratch(psf, false));
    const bool fp64 = psf ? psf->fp64 : pl->fp64;
    const size_t rs = fp64 ? 8 : 4;
    const int64_t nx = psf ? psf->nx : pl->nx, ny = psf ? psf->ny : pl->ny, nc = psf ? psf->n_chan : pl->n_chan;
    const size_t vec = scratch_round((size_t)nc * nx * ny * rs);
    const size_t loop = scratch_round(sizeof(CGState)) + scratch_round(2 * (size_t)red_blocks(nc * nx * ny) * 8) +
                        scratch_round(2 * sizeof(double)) + 3 * vec;
    const size_t apply = std::max(prior ? periodic_conv_scratch(nc, nx, ny, fp64) : size_t(0),
                                  psf ? rnr_approx_scratch(psf, 1) : rnr_exact_scratch(pl));
    return 2 * vec + (prior ? vec : 0) + loop + apply;
}

template <typename T>
void cg_solve(const fr_plan *pl, const fr_psf *psf, const T *weight, const T *inv_power, const T *diag, const T *b,
              T *x, int maxiter, double rtol, double *hist, int *iters_done, hipStream_t st) {
    if (cg_fused_applies(psf, inv_power != nullptr)) {
        cg_solve_psf_fused<T>(psf, inv_power, diag, b, x, maxiter, rtol, hist, iters_done, st);
        return;
    }
    const int64_t nx = psf ? psf->nx : pl->nx, ny = psf ? psf->ny : pl->ny;
    const int64_t nc = psf ? psf->n_chan : pl->n_chan;
    const int64_t n = nc * nx * ny;
    const Ctx &ctx = psf ? *psf->ctx : *pl->ctx;
    Scratch t(n * sizeof(T), st), u(n * sizeof(T), st);
    Scratch pr;
    if (inv_power) pr = Scratch(n * sizeof(T), st);
    cg_run<T>(n, b, x, maxiter, rtol, hist, iters_done, st, [&](const T *p, T *Ap) {
        // A p = D R' D p + S^-1 p
        if (inv_power) periodic_conv<T>(ctx, p, pr.as<T>(), nc, nx, ny, inv_power, 1, 0, st);
        const T *prior = inv_power ? pr.as<T>() : nullptr;
        if (psf) {
            apply_rnr_approx_ex<T>(psf, p, diag, Ap, diag, prior, 1, st);
        } else {
            const T *src = p;
            if (diag) {
                map_async(DiagMul<T>{diag, p, t.as<T>()}, n, st);
                src = t.as<T>();
            }
            apply_rnr_exact<T>(pl, weight, src, u.as<T>(), 1, st);
            map_async(DiagMulAdd<T>{diag, u.as<T>(), prior, Ap}, n, st);
        }
    });
}

// ------------------------------------------------------------------ MGVI
// Minor-cycle posterior in standardised coordinates xi (log-sky s = A xi, A =
// F^-1 sqrt(P) F, the exponentiated Gaussian process of the prior), FAST
// likelihood: Fisher metric M = 1 + A D R' N'^-1 R' D A with D = diag(exp s).
enum { kConvMul = 0, kConvDiv = 1, kConvMulSqrt = 2, kConvDivSqrt = 3 };

template <typename T> struct MgviOp {
    const fr_psf *psf;
    const T *power, *diag;
    int64_t nx, ny, nc, n;
    // y = x + A D R' N'^-1 R' D A x  (u1, u2 scratch of n values)
    void metric(const T *x, T *y, T *u1, T *u2, hipStream_t st) const {
        const Ctx &ctx = *psf->ctx;
        periodic_conv_ex<T>(ctx, x, nullptr, u1, nullptr, nullptr, nc, nx, ny, power, 1, kConvMulSqrt, st);
        apply_rnr_approx_ex<T>(psf, u1, diag, u2, nullptr, nullptr, 1, st);
        periodic_conv_ex<T>(ctx, u2, nullptr, u1, nullptr, nullptr, nc, nx, ny, psf->KN.as<T>(), (int)nc, kConvDiv,
                            st);
        apply_rnr_approx_ex<T>(psf, u1, nullptr, u2, diag, nullptr, 1, st);
        periodic_conv_ex<T>(ctx, u2, nullptr, y, nullptr, x, nc, nx, ny, power, 1, kConvMulSqrt, st);
    }
};

template <typename T>
void mgvi_metric_apply(const fr_psf *psf, const T *power, const T *diag, const T *x, T *y, hipStream_t st) {
    const int64_t n = psf->n_chan * psf->nx * psf->ny;
    MgviOp<T> op{psf, power, diag, psf->nx, psf->ny, psf->n_chan, n};
    Scratch u1(n * sizeof(T), st), u2(n * sizeof(T), st);
    op.metric(x, y, u1.as<T>(), u2.as<T>(), st);
}

// xi = eta0 + A D R' N'^-1/2 eta1: covariance M for white eta0, eta1
template <typename T>
void mgvi_draw(const fr_psf *psf, const T *power, const T *diag, const T *eta0, const T *eta1, T *xi,
               hipStream_t st) {
    const int64_t nx = psf->nx, ny = psf->ny, nc = psf->n_chan, n = nc * nx * ny;
    const Ctx &ctx = *psf->ctx;
    Scratch u1(n * sizeof(T), st), u2(n * sizeof(T), st);
    periodic_conv_ex<T>(ctx, eta1, nullptr, u1.as<T>(), nullptr, nullptr, nc, nx, ny, psf->KN.as<T>(), (int)nc,
                        kConvDivSqrt, st);
    apply_rnr_approx_ex<T>(psf, u1.as<T>(), nullptr, u2.as<T>(), diag, nullptr, 1, st);
    periodic_conv_ex<T>(ctx, u2.as<T>(), nullptr, xi, nullptr, eta0, nc, nx, ny, power, 1, kConvMulSqrt, st);
}

// M x = b by CG (b = an mgvi_draw gives the sample offset x ~ N(0, M^-1))
template <typename T>
void mgvi_solve(const fr_psf *psf, const T *power, const T *diag, const T *b, T *x, int maxiter, double rtol,
                double *hist, int *iters_done, hipStream_t st) {
    const int64_t n = psf->n_chan * psf->nx * psf->ny;
    MgviOp<T> op{psf, power, diag, psf->nx, psf->ny, psf->n_chan, n};
    Scratch u1(n * sizeof(T), st), u2(n * sizeof(T), st);
    cg_run<T>(n, b, x, maxiter, rtol, hist, iters_done, st,
              [&](const T *p, T *Ap) { op.metric(p, Ap, u1.as<T>(), u2.as<T>(), st); });
}

template void cg_solve<float>(const fr_plan *, const fr_psf *, const float *, const float *, const float *,
                              const float *, float *, int, double, double *, int *, hipStream_t);
template void cg_solve<double>(const fr_plan *, const fr_psf *, const double *, const double *, const double *,
                               const double *, double *, int, double, double *, int *, hipStream_t);
template void mgvi_metric_apply<float>(const fr_psf *, const float *, const float *, const float *, float *,
                                       hipStream_t);
template void mgvi_metric_apply<double>(const fr_psf *, const double *, const double *, const double *, double *,
                                        hipStream_t);
template void mgvi_draw<float>(const fr_psf *, const float *, const float *, const float *, const float *, float *,
                               hipStream_t);
template void mgvi_draw<double>(const fr_psf *, const double *, const double *, const double *, const double *,
                                double *, hipStream_t);
template void mgvi_solve<float>(const fr_psf *, const float *, const float *, const float *, float *, int, double,
                                double *, int *, hipStream_t);
template void mgvi_solve<double>(const fr_psf *, const double *, const double *, const double *, double *, int,
                                 double, double *, int *, hipStream_t);

}  // namespace frmi
