// Conjugate gradients on A x = D_s R' D_s x + S^-1 x = b: the solve MGVI uses to
// apply the inverse metric in the minor cycle (Sec. 3.3.5).  Hestenes-Stiefel
// recurrences with x0 = 0 and no preconditioner.
//
// Vectors are in the plan/PSF precision; <r, r>, <p, A p>, alpha and beta are
// double precision scalars that live on the device.  Every kernel reads them
// from device memory, so the host enqueues `maxiter` iterations without ever
// synchronising; once ||r|| <= rtol ||b|| a device flag turns the remaining
// update kernels into no-ops.
#include "conv.h"
#include "elementwise.h"
#include "objects.h"

namespace frmi {

struct CGState {
    double rr;     // <r, r>
    double pAp;    // <p, A p>
    double beta;
    double stop;   // rtol ||b||
    int done;
    int iters;
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

__global__ void k_cg_start(CGState *st, const double *rr_partials, int nparts, double rtol, int maxiter,
                           double *hist) {
    if (threadIdx.x != 0) return;
    double s = 0;
    for (int k = 0; k < nparts; ++k) s += rr_partials[k];
    st->rr = s;
    st->stop = rtol * sqrt(s);
    st->iters = 0;
    st->done = (s == 0.0 || maxiter == 0) ? 1 : 0;
    st->beta = 0;
    hist[0] = sqrt(s);
}

struct ZeroU32 {
    unsigned *p;
    __device__ void operator()(int64_t i) const { p[i] = 0u; }
};

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

// The last block to finish a reduction adds the per-block partials in block
// order (deterministic) and resets the arrival counter for the next use.
__device__ __forceinline__ bool arrive_last(unsigned *counter) {
    __shared__ bool last;
    __threadfence();
    if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
    __syncthreads();
    return last;
}

// Called by every thread of the last block: the partials are fetched in
// parallel (device-coherent loads), then added by thread 0 in block order.
__device__ __forceinline__ double sum_partials(const double *partials, int n) {
    __shared__ double sh[kRedBlocksPerImage];
    for (int k = threadIdx.x; k < n; k += blockDim.x)
        sh[k] = __hip_atomic_load(partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < n; ++k) s += sh[k];
    return s;  // valid in thread 0
}

// <p, A p> into st->pAp
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_dot_pAp(CGState *__restrict__ st, const T *__restrict__ p,
                                                            const T *__restrict__ Ap, int64_t n,
                                                            double *__restrict__ partials, unsigned *counter) {
    if (st->done) return;
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads)
        s += (double)p[i] * (double)Ap[i];
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
    if (arrive_last(counter)) {
        const double t = sum_partials(partials, gridDim.x);
        if (threadIdx.x == 0) {
            st->pAp = t;
            *counter = 0;
        }
    }
}

// x += alpha p, r -= alpha A p; the last block forms <r, r>, beta, the history
// entry and the stopping flag
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_cg_step(CGState *__restrict__ st, T *__restrict__ x,
                                                         T *__restrict__ r, const T *__restrict__ p,
                                                         const T *__restrict__ Ap, int64_t n,
                                                         double *__restrict__ partials, unsigned *counter, int k,
                                                         double *__restrict__ hist) {
    if (st->done) return;
    const T a = (T)(st->rr / st->pAp);
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRedThreads) {
        x[i] += a * p[i];
        const T rv = r[i] - a * Ap[i];
        r[i] = rv;
        s += (double)rv * (double)rv;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
    if (arrive_last(counter)) {
        const double rr = sum_partials(partials, gridDim.x);
        if (threadIdx.x == 0) {
            hist[k + 1] = sqrt(rr);
            st->beta = rr / st->rr;
            st->rr = rr;
            st->iters = k + 1;
            if (sqrt(rr) <= st->stop) st->done = 1;
            *counter = 0;
        }
    }
}

template <typename T>
__global__ void k_cg_update_p(const CGState *__restrict__ st, T *__restrict__ p, const T *__restrict__ r, int64_t n) {
    if (st->done) return;
    const T beta = (T)st->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * p[i];
}

__global__ void k_cg_report(const CGState *st, int *iters_done) {
    if (threadIdx.x == 0) *iters_done = st->iters;
}

template <typename T>
void cg_solve(const fr_plan *pl, const fr_psf *psf, const T *weight, const T *inv_power, const T *diag, const T *b,
              T *x, int maxiter, double rtol, double *hist, int *iters_done, hipStream_t st) {
    const int64_t nx = psf ? psf->nx : pl->nx, ny = psf ? psf->ny : pl->ny;
    const int64_t nc = psf ? psf->n_chan : pl->n_chan;
    const int64_t n = nc * nx * ny;
    const Ctx &ctx = psf ? *psf->ctx : *pl->ctx;
    Scratch state(sizeof(CGState) + 64, st);
    Scratch partials((size_t)kRedBlocksPerImage * sizeof(double), st);
    unsigned *counter = reinterpret_cast<unsigned *>(state.as<char>() + sizeof(CGState));
    map_async(ZeroU32{counter}, 1, st);
    Scratch r(n * sizeof(T), st), p(n * sizeof(T), st), Ap(n * sizeof(T), st), t(n * sizeof(T), st),
        u(n * sizeof(T), st);
    Scratch pr;
    if (inv_power) pr = Scratch(n * sizeof(T), st);
    CGState *S = state.as<CGState>();
    map_async(CGInit<T>{b, x, r.as<T>(), p.as<T>()}, n, st);
    k_dot_partials<T><<<dim3(kRedBlocksPerImage, 1), kRedThreads, 0, st>>>(r.as<T>(), nullptr, n,
                                                                         partials.as<double>());
    LAUNCH_CHECK();
    k_cg_start<<<1, 64, 0, st>>>(S, partials.as<double>(), kRedBlocksPerImage, rtol, maxiter, hist);
    LAUNCH_CHECK();
    for (int k = 0; k < maxiter; ++k) {
        // A p = D R' D p + S^-1 p
        if (inv_power) periodic_conv<T>(ctx, p.as<T>(), pr.as<T>(), nc, nx, ny, inv_power, 1, 0, st);
        const T *prior = inv_power ? pr.as<T>() : nullptr;
        if (psf) {
            apply_rnr_approx_ex<T>(psf, p.as<T>(), diag, Ap.as<T>(), diag, prior, 1, st);
        } else {
            const T *src = p.as<T>();
            if (diag) {
                map_async(DiagMul<T>{diag, p.as<T>(), t.as<T>()}, n, st);
                src = t.as<T>();
            }
            apply_rnr_exact<T>(pl, weight, src, u.as<T>(), 1, st);
            map_async(DiagMulAdd<T>{diag, u.as<T>(), prior, Ap.as<T>()}, n, st);
        }
        k_cg_dot_pAp<T><<<dim3(kRedBlocksPerImage), kRedThreads, 0, st>>>(S, p.as<T>(), Ap.as<T>(), n,
                                                                          partials.as<double>(), counter);
        LAUNCH_CHECK();
        k_cg_step<T><<<dim3(kRedBlocksPerImage), kRedThreads, 0, st>>>(S, x, r.as<T>(), p.as<T>(), Ap.as<T>(), n,
                                                                       partials.as<double>(), counter, k, hist);
        LAUNCH_CHECK();
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
        k_cg_update_p<T><<<dim3((unsigned)blocks), 256, 0, st>>>(S, p.as<T>(), r.as<T>(), n);
        LAUNCH_CHECK();
    }
    k_cg_report<<<1, 64, 0, st>>>(S, iters_done);
    LAUNCH_CHECK();
}

template void cg_solve<float>(const fr_plan *, const fr_psf *, const float *, const float *, const float *,
                              const float *, float *, int, double, double *, int *, hipStream_t);
template void cg_solve<double>(const fr_plan *, const fr_psf *, const double *, const double *, const double *,
                               const double *, double *, int, double, double *, int *, hipStream_t);

}  // namespace frmi
