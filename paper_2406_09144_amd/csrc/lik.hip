// Exact R' = R^+ N^-1 R (major cycle, Sec. 3.3.4) and the likelihood
// Hamiltonians with their log-sky gradients: eq. ham (Sec. 3.1.2, through the
// exact operators) and eq. ham_new (Sec. 3.3.1, through the PSF and noise-kernel
// convolutions of Sec. 3.3.2-3.3.3).
#include "conv.h"
#include "elementwise.h"
#include "objects.h"

namespace frmi {

size_t rnr_exact_scratch(const fr_plan *pl) {
    const size_t cs = pl->fp64 ? sizeof(double2) : sizeof(float2);
    return scratch_round((size_t)pl->n_vis * cs) + std::max(degrid_scratch(pl), grid_scratch(pl));
}

size_t lik_scratch(const fr_plan *pl, const fr_psf *psf, int mode, int64_t B, bool prior) {
    const bool fp64 = mode == FR_LIK_FAST ? psf->fp64 : pl->fp64;
    const size_t rs = fp64 ? 8 : 4;
    const int64_t nx = mode == FR_LIK_FAST ? psf->nx : pl->nx, ny = mode == FR_LIK_FAST ? psf->ny : pl->ny;
    const int64_t nc = mode == FR_LIK_FAST ? psf->n_chan : pl->n_chan;
    const size_t n_all = (size_t)B * nc * nx * ny;
    const size_t per = scratch_round((size_t)std::max<int64_t>(B, 1) * kRedMaxBlocks * sizeof(double)) +
                       2 * scratch_round(n_all * rs);
    const size_t yper = periodic_conv_scratch(B * nc, nx, ny, fp64);
    const size_t body = mode == FR_LIK_FAST
                            ? scratch_round(n_all * rs) + std::max(rnr_approx_scratch(psf, B), yper)
                            : rnr_exact_scratch(pl);
    return per + std::max(body, prior ? scratch_round(n_all * rs) + yper : size_t(0));
}

// R^+ N^-1 R x: the degridded values of every record, times its weight, go back
// to the spread in record order (coalesced stores and loads, no gathers; the
// centring phase and the conjugation of w < 0 records cancel between R and R^+)
template <typename T>
void apply_rnr_exact(const fr_plan *pl, const T *weight, const T *x, T *y, int64_t B, hipStream_t st) {
    const int64_t n_img = pl->n_chan * pl->nx * pl->ny;
    Scratch vis((size_t)pl->n_vis * sizeof(c2<T>), st);
    for (int64_t b = 0; b < B; ++b) {
        degrid<T>(pl, x + b * n_img, vis.as<c2<T>>(), st, weight, true);
        grid<T>(pl, vis.as<c2<T>>(), nullptr, y + b * n_img, st, true);
    }
}

// I = exp(s) + i_fixed (i_fixed broadcast over the batch)
template <typename T> struct SkyFromLog {
    const T *s, *ifix;
    T *I;
    int64_t n_img;
    double inv_n;
    __device__ void operator()(int64_t q) const {
        T v = exp(s[q]);
        if (ifix) v += ifix[mod_nonneg(q, n_img, inv_n)];
        I[q] = v;
    }
};

// r = d - t (d broadcast over the batch), in place on t
template <typename T> struct Residual {
    const T *d;
    T *t;
    int64_t n_img;
    double inv_n;
    __device__ void operator()(int64_t q) const { t[q] = d[mod_nonneg(q, n_img, inv_n)] - t[q]; }
};

// g = sign * exp(s) * u (+ prior)
template <typename T> struct GradFromLog {
    const T *s, *u, *prior;
    T *g;
    T sign;
    __device__ void operator()(int64_t q) const {
        T v = sign * exp(s[q]) * u[q];
        if (prior) v += prior[q];
        g[q] = v;
    }
};

// residual in visibility space: res = w (model - V), partial sums of w |model - V|^2
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_vis_residual(c2<T> *__restrict__ model, const c2<T> *__restrict__ V,
                                                              const T *__restrict__ w, int64_t n,
                                                              double *__restrict__ partials) {
    double s = grid_stride_sum(n, [&](int64_t i) {
        const c2<T> m = model[i], v = V[i];
        const T wt = w ? w[i] : T(1);
        const T dx = m.x - v.x, dy = m.y - v.y;
        model[i] = mk<T>(wt * dx, wt * dy);
        return (double)wt * ((double)dx * dx + (double)dy * dy);
    });
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
void likelihood_grad(const fr_plan *pl, const fr_psf *psf, int mode, const T *s, const T *i_fixed, const void *data,
                     const T *weight, const T *inv_power, int64_t B, T *grad, double *H, hipStream_t st) {
    const int64_t nx = mode == FR_LIK_FAST ? psf->nx : pl->nx;
    const int64_t ny = mode == FR_LIK_FAST ? psf->ny : pl->ny;
    const int64_t nc = mode == FR_LIK_FAST ? psf->n_chan : pl->n_chan;
    const int64_t n_img = nc * nx * ny;  // one sample
    const int64_t n_all = B * n_img;
    const Ctx &ctx = mode == FR_LIK_FAST ? *psf->ctx : *pl->ctx;
    Scratch partials((size_t)std::max<int64_t>(B, 1) * kRedMaxBlocks * sizeof(double), st);
    Scratch Ib((size_t)n_all * sizeof(T), st);
    Scratch ub((size_t)n_all * sizeof(T), st);
    map_async(SkyFromLog<T>{s, i_fixed, Ib.as<T>(), n_img, 1.0 / (double)n_img}, n_all, st);
    if (mode == FR_LIK_FAST) {
        FR_REQUIRE(psf->KN.p, "the PSF object has no noise kernel");
        Scratch tb((size_t)n_all * sizeof(T), st);
        // r = d - R' I
        apply_rnr_approx<T>(psf, Ib.as<T>(), tb.as<T>(), B, st);
        map_async(Residual<T>{(const T *)data, tb.as<T>(), n_img, 1.0 / (double)n_img}, n_all, st);
        // q = N'^-1 r  (into Ib, no longer needed)
        periodic_conv<T>(ctx, tb.as<T>(), Ib.as<T>(), B * nc, nx, ny, psf->KN.as<T>(), (int)nc, 1, st);
        // H = 1/2 <r, q>
        batched_dot<T>(tb.as<T>(), Ib.as<T>(), n_img, B, 0.5, 0, H, partials.as<double>(), st);
        // g = -exp(s) R' q
        apply_rnr_approx<T>(psf, Ib.as<T>(), ub.as<T>(), B, st);
    } else {
        Scratch vis((size_t)pl->n_vis * sizeof(c2<T>), st);
        const int nblk = red_blocks(pl->n_vis);
        for (int64_t b = 0; b < B; ++b) {
            degrid<T>(pl, Ib.as<T>() + b * n_img, vis.as<c2<T>>(), st);
            k_vis_residual<T><<<dim3(nblk), kRedThreads, 0, st>>>(vis.as<c2<T>>(), (const c2<T> *)data, weight,
                                                                  pl->n_vis, partials.as<double>());
            LAUNCH_CHECK();
            k_finish_sums<<<1, kRedThreads, 0, st>>>(partials.as<double>(), nblk, 0.5, 0, H + b);
            LAUNCH_CHECK();
            grid<T>(pl, vis.as<c2<T>>(), nullptr, ub.as<T>() + b * n_img, st);
        }
    }
    T *prior = nullptr;
    Scratch sp;
    if (inv_power) {
        sp = Scratch((size_t)n_all * sizeof(T), st);
        periodic_conv<T>(ctx, s, sp.as<T>(), B * nc, nx, ny, inv_power, 1, 0, st);
        batched_dot<T>(s, sp.as<T>(), n_img, B, 0.5, 1, H, partials.as<double>(), st);
        prior = sp.as<T>();
    }
    map_async(GradFromLog<T>{s, ub.as<T>(), prior, grad, T(mode == FR_LIK_FAST ? -1 : 1)}, n_all, st);
}

template void apply_rnr_exact<float>(const fr_plan *, const float *, const float *, float *, int64_t, hipStream_t);
template void apply_rnr_exact<double>(const fr_plan *, const double *, const double *, double *, int64_t,
                                      hipStream_t);
template void likelihood_grad<float>(const fr_plan *, const fr_psf *, int, const float *, const float *,
                                     const void *, const float *, const float *, int64_t, float *, double *,
                                     hipStream_t);
template void likelihood_grad<double>(const fr_plan *, const fr_psf *, int, const double *, const double *,
                                      const void *, const double *, const double *, int64_t, double *, double *,
                                      hipStream_t);

}  // namespace frmi
