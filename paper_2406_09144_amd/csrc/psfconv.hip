// PSF-convolution response R' ~ I_PSF * (Sec. 3.3.2) and periodic convolutions
// (noise kernel, Sec. 3.3.3; prior covariance) on the GPU.
#include "conv.h"
#include "fftk.h"
#include "objects.h"
#include "profiler.h"

namespace frmi {

// y = D P^+ irfft2(K_R rfft2(P D x)): x padded into the top-left nx x ny block of
// the px x py grid of the response kernel (2nx x 2ny, or n + h per axis for a
// reduced support).  Only the nx non-zero rows are transformed along y and only
// the nx wanted rows are kept after the column pass.
// y = d_out D P^+ irfft2(K_R rfft2(P D d_in x)) + add, every extra factor optional:
// the diagonal metric factors and the prior term of CG fused into the first and
// last pass.  The half-spectrum buffer (and, for columns of 8192 points or more,
// the four-step column pass's buffer after it) comes from the stream's arena, or
// from `ws` (at least rnr_approx_scratch bytes, 256-byte aligned) when that is
// given; every element is written before it is read, so it needs no clearing.
template <typename T>
void apply_rnr_approx_ex(const fr_psf *psf, const T *x, const T *d_in, T *y, const T *d_out, const T *add,
                         int64_t B, hipStream_t st, void *ws) {
    const int64_t nx = psf->nx, ny = psf->ny, nc = psf->n_chan;
    const int64_t n_img = B * nc;
    if (n_img == 0) return;
    ConvGeom g;
    g.n_img = n_img;
    g.rows_in = (int)nx;
    g.rows_out = (int)nx;
    g.n_in_cols = (int)ny;
    g.n_out_cols = (int)ny;
    FR_REQUIRE(split_len(psf->py / 2, &g.odd_M, &g.log2M) && split_len(psf->px, &g.odd_Lc, &g.log2Lc),
               "padded kernel sizes must be 2^p, 3 2^p or 5 2^p");
    const int64_t M = g.M();
    Scratch Yarena;
    if (!ws) Yarena = Scratch((size_t)n_img * nx * M * sizeof(c2<T>), st);
    c2<T> *const Yp = ws ? (c2<T> *)ws : Yarena.as<c2<T>>();
    const T *a = psf->nfac.as<T>();
    with_odd(g.odd_M, [&](auto odd) {
        ProfScope prof("psfconv_rows_r2c", st);
        launch_rfft_rows<T, decltype(odd)::value>(*psf->ctx, g, ProDiagScaled<T>{x, d_in, a, (int)nx, (int)ny},
                                                  Yp, st);
    });
    const T scale = T(1) / (T(g.Lc()) * T(M));
    with_odd(g.odd_Lc, [&](auto odd) {
        ProfScope prof("psfconv_cols", st);
        void *zws = ws ? (char *)ws + scratch_round((size_t)n_img * nx * M * sizeof(c2<T>)) : nullptr;
        launch_conv_cols<T, decltype(odd)::value>(*psf->ctx, g, Yp, psf->KR.as<T>(), (int)nc, 0, scale,
                                                  st, nullptr, INT64_MAX, nullptr, zws);
    });
    with_odd(g.odd_M, [&](auto odd) {
        ProfScope prof("psfconv_rows_c2r", st);
        launch_irfft_rows<T, decltype(odd)::value>(*psf->ctx, g, EpiDiagScaledAdd<T>{y, d_out, a, add, (int)nx, (int)ny},
                                                   Yp, st);
    });
}

// four-step buffer of a column pass of Lc points over n_img images of M packed columns
static size_t cols_extra(int64_t n_img, int64_t Lc, int64_t M, size_t cs) {
    int odd = 1, l = 0;
    if (!split_len(Lc, &odd, &l)) return 0;
    return conv4_applies((int)Lc, odd, (int)M, cs) ? scratch_round(conv4_scratch(n_img, (int)Lc, (int)M, cs)) : 0;
}

size_t rnr_approx_scratch(const fr_psf *psf, int64_t B) {
    const size_t cs = psf->fp64 ? sizeof(double2) : sizeof(float2);
    const int64_t n_img = B * psf->n_chan, M = psf->py / 2;
    return scratch_round((size_t)n_img * psf->nx * M * cs) + cols_extra(n_img, psf->px, M, cs);
}

size_t periodic_conv_scratch(int64_t n_img, int64_t nx, int64_t ny, bool fp64) {
    const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
    return scratch_round((size_t)n_img * nx * (ny / 2) * cs) + cols_extra(n_img, nx, ny / 2, cs);
}

template <typename T>
void apply_rnr_approx(const fr_psf *psf, const T *x, T *y, int64_t B, hipStream_t st) {
    apply_rnr_approx_ex<T>(psf, x, nullptr, y, nullptr, nullptr, B, st);
}

// y = d_out * irfft2(f(K) rfft2(d_in * x)) + add on the periodic nx x ny grid,
// f(K) as kernel_factor(mode); every extra factor optional (NULL).
template <typename T>
void periodic_conv_ex(const Ctx &ctx, const T *x, const T *d_in, T *y, const T *d_out, const T *add,
                      int64_t n_img, int64_t nx, int64_t ny, const T *K, int nk, int mode, hipStream_t st) {
    if (n_img == 0) return;
    ConvGeom g;
    g.n_img = n_img;
    g.rows_in = (int)nx;
    g.rows_out = (int)nx;
    g.n_in_cols = (int)ny;
    g.n_out_cols = (int)ny;
    g.log2M = ilog2(ny / 2);
    g.log2Lc = ilog2(nx);
    Scratch Y((size_t)n_img * nx * (ny / 2) * sizeof(c2<T>), st);
    {
        ProfScope prof("pconv_rows_r2c", st);
        launch_rfft_rows<T>(ctx, g, ProDiagScaled<T>{x, d_in, nullptr, (int)nx, (int)ny}, Y.as<c2<T>>(), st);
    }
    const T scale = T(1) / (T(nx) * T(ny / 2));
    {
        ProfScope prof("pconv_cols", st);
        launch_conv_cols<T>(ctx, g, Y.as<c2<T>>(), K, nk, mode, scale, st);
    }
    ProfScope prof("pconv_rows_c2r", st);
    launch_irfft_rows<T>(ctx, g, EpiDiagScaledAdd<T>{y, d_out, nullptr, add, (int)nx, (int)ny}, Y.as<c2<T>>(), st);
}

// y = irfft2(f(K) rfft2(x)) on the periodic nx x ny grid (f as kernel_factor:
// mode 0 K, 1 1/K); K is [nk][nx][ny/2 + 1], image g uses K[g % nk].
template <typename T>
void periodic_conv(const Ctx &ctx, const T *x, T *y, int64_t n_img, int64_t nx, int64_t ny, const T *K, int nk,
                   int mode, hipStream_t st) {
    periodic_conv_ex<T>(ctx, x, nullptr, y, nullptr, nullptr, n_img, nx, ny, K, nk, mode, st);
}

template <typename T>
void fft2_inplace(const Ctx &ctx, c2<T> *data, int64_t batch, int64_t n0, int64_t n1, int sign, hipStream_t st) {
    int o0 = 1, l0 = 0, o1 = 1, l1 = 0;
    FR_REQUIRE(split_len(n0, &o0, &l0) && split_len(n1, &o1, &l1), "FFT sizes must be 2^p, 3 2^p or 5 2^p");
    with_odd(o1, [&](auto odd) {
        launch_fft_rows<T, RowLoad<T>, RowStore<T>, decltype(odd)::value>(ctx, RowLoad<T>{data, n1},
                                                                          RowStore<T>{data, n1}, batch * n0, l1, sign,
                                                                          st);
    });
    with_odd(o0, [&](auto odd) {
        launch_fft_cols<T, MatLoad<T>, MatStore<T>, decltype(odd)::value>(
            ctx, MatLoad<T>{data, n0 * n1, (int)n1}, MatStore<T>{data, n0 * n1, (int)n1}, batch, (int)n1, l0, (int)n0,
            (int)n0, sign, st);
    });
}

template void apply_rnr_approx_ex<float>(const fr_psf *, const float *, const float *, float *, const float *,
                                         const float *, int64_t, hipStream_t, void *);
template void apply_rnr_approx_ex<double>(const fr_psf *, const double *, const double *, double *, const double *,
                                          const double *, int64_t, hipStream_t, void *);
template void apply_rnr_approx<float>(const fr_psf *, const float *, float *, int64_t, hipStream_t);
template void apply_rnr_approx<double>(const fr_psf *, const double *, double *, int64_t, hipStream_t);
template void periodic_conv<float>(const Ctx &, const float *, float *, int64_t, int64_t, int64_t, const float *, int,
                                   int, hipStream_t);
template void periodic_conv<double>(const Ctx &, const double *, double *, int64_t, int64_t, int64_t, const double *,
                                    int, int, hipStream_t);
template void periodic_conv_ex<float>(const Ctx &, const float *, const float *, float *, const float *,
                                      const float *, int64_t, int64_t, int64_t, const float *, int, int, hipStream_t);
template void periodic_conv_ex<double>(const Ctx &, const double *, const double *, double *, const double *,
                                       const double *, int64_t, int64_t, int64_t, const double *, int, int,
                                       hipStream_t);
template void fft2_inplace<float>(const Ctx &, float2 *, int64_t, int64_t, int64_t, int, hipStream_t);
template void fft2_inplace<double>(const Ctx &, double2 *, int64_t, int64_t, int64_t, int, hipStream_t);

}  // namespace frmi
