// Correlated-field amplitude model of the diffuse-emission prior (the inferred
// power spectrum of the exponentiated Gaussian process, Sec. 3.1.1, with the
// hyperparameters of the prior-parameter appendices: zero-mode offset, zero-mode
// standard deviation, fluctuations, average log-log slope, flexibility and
// asperity).
//
// Reading of the model (the paper defers its definition to earlier work):
//   * zero-mode std, fluctuations, flexibility and asperity are lognormal with
//     the given mean and standard deviation, x = exp(mu + sigma xi) with
//     sigma^2 = ln(1 + std^2 / mean^2), mu = ln(mean) - sigma^2 / 2 (a mean of 0
//     gives 0); the average slope is normal;
//   * over the distinct non-zero |k| of the grid, at t = ln|k| ascending with
//     steps d_j (d_0 = 0), the local slope v_j = flex sum_{i<=j} sqrt(d_i) xi_v_i
//     is a Wiener process, y_j = sum_{i<=j} [(v_i-1 + v_i) d_i / 2 +
//     flex asp sqrt(d_i) xi_y_i] integrates it with a rougher Wiener part, and
//     logA_j = slope (t_j - t_0) + y_j - y_J (t_j - t_0) / (t_J - t_0);
//   * P_j = fluct^2 N A_j^2 / sum_j mult_j A_j^2 for k != 0 (mult_j: frequencies
//     of the full grid in bin j), P(0) = zm^2 N, so the field without its zero
//     mode has variance fluct^2 and the zero mode zm^2;
//   * log-sky = offset + F^-1 sqrt(P) F xi_field.
//
// The scans run in one workgroup in FP64 (a chunk of bins per thread, a block
// scan of the chunk sums, then the chunk's running values), so the result
// depends only on the input; the power is written in the requested precision.
#include <cmath>
#include <numeric>

#include "cfbins.h"
#include "conv.h"
#include "elementwise.h"
#include "objects.h"

namespace frmi {

struct CFPrior {
    double v[11];  // offset, zm mean/std, fluct mean/std, slope mean/std, flex mean/std, asp mean/std
};

constexpr int kCFThreads = 1024;

__device__ __forceinline__ double lognormal_moments(double mean, double sd, double xi) {
    if (mean == 0.0) return 0.0;
    const double s2 = log1p((sd / mean) * (sd / mean));
    return exp(log(mean) - 0.5 * s2 + sqrt(s2) * xi);
}

// Exclusive scan of one value per thread across the workgroup (FP64, fixed order);
// returns this thread's exclusive prefix; *total gets the sum (all threads).
__device__ double block_exclusive_scan(double v, double *total) {
    __shared__ double sh[kCFThreads];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kCFThreads; off <<= 1) {
        const double add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const double incl = sh[threadIdx.x];
    *total = sh[kCFThreads - 1];
    __syncthreads();
    return incl - v;
}

__device__ double block_reduce(double v, bool is_max) {
    __shared__ double sh[kCFThreads / 64];
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_down(v, o, 64);
        v = is_max ? fmax(v, w) : v + w;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = sh[0];
    for (int k = 1; k < kCFThreads / 64; ++k) t = is_max ? fmax(t, sh[k]) : t + sh[k];
    __syncthreads();
    return t;
}

// One workgroup: hyperparameters, the two Wiener scans, detrending, normalisation.
// t, d, mult: [J]; work: [2 J] (v, then logA); P_bin: [J]; P0: [1].
__global__ __launch_bounds__(kCFThreads) void k_cf_spectrum(CFPrior pr, int64_t J, double n_pix,
                                                            const double *__restrict__ t,
                                                            const double *__restrict__ d,
                                                            const double *__restrict__ mult,
                                                            const double *__restrict__ xi_h,
                                                            const double *__restrict__ xi_v,
                                                            const double *__restrict__ xi_y, double *__restrict__ v,
                                                            double *__restrict__ logA, double *__restrict__ P_bin,
                                                            double *__restrict__ P0) {
    const double zm = lognormal_moments(pr.v[1], pr.v[2], xi_h[0]);
    const double fluct = lognormal_moments(pr.v[3], pr.v[4], xi_h[1]);
    const double slope = pr.v[5] + pr.v[6] * xi_h[2];
    const double flex = lognormal_moments(pr.v[7], pr.v[8], xi_h[3]);
    const double asp = lognormal_moments(pr.v[9], pr.v[10], xi_h[4]);
    const int64_t chunk = (J + kCFThreads - 1) / kCFThreads;
    const int64_t b0 = min<int64_t>(J, (int64_t)threadIdx.x * chunk), b1 = min<int64_t>(J, b0 + chunk);
    double total = 0.0;
    // v: the local slope (Wiener process)
    double s = 0.0;
    for (int64_t j = b0; j < b1; ++j) s += flex * sqrt(d[j]) * xi_v[j];
    double run = block_exclusive_scan(s, &total);
    for (int64_t j = b0; j < b1; ++j) {
        run += flex * sqrt(d[j]) * xi_v[j];
        v[j] = run;
    }
    __syncthreads();  // v of the neighbouring chunk is read below
    // y: its integral plus the rough part
    auto y_inc = [&](int64_t j) {
        const double vp = j > 0 ? v[j - 1] : 0.0;
        return 0.5 * (vp + v[j]) * d[j] + flex * asp * sqrt(d[j]) * xi_y[j];
    };
    s = 0.0;
    for (int64_t j = b0; j < b1; ++j) s += y_inc(j);
    double yJ = 0.0;
    run = block_exclusive_scan(s, &yJ);
    const double t0 = t[0], span = t[J - 1] - t[0];
    double mx = -INFINITY;
    for (int64_t j = b0; j < b1; ++j) {
        run += y_inc(j);
        const double frac = span > 0 ? (t[j] - t0) / span : 0.0;
        const double la = slope * (t[j] - t0) + run - yJ * frac;
        logA[j] = la;
        mx = fmax(mx, la);
    }
    mx = block_reduce(mx, true);
    double acc = 0.0;
    for (int64_t j = b0; j < b1; ++j) acc += mult[j] * exp(2.0 * (logA[j] - mx));
    const double norm = block_reduce(acc, false);
    const double scale = fluct * fluct * n_pix / norm;
    for (int64_t j = b0; j < b1; ++j) P_bin[j] = scale * exp(2.0 * (logA[j] - mx));
    if (threadIdx.x == 0) *P0 = zm * zm * n_pix;
}

// power on the r2c half spectrum [nx][ny/2 + 1] from the per-bin values
template <typename T> struct CFScatter {
    const int32_t *bin;
    const double *P_bin, *P0;
    T *out;
    __device__ void operator()(int64_t q) const {
        const int32_t b = bin[q];
        out[q] = (T)(b < 0 ? *P0 : P_bin[b]);
    }
};

void cf_build(fr_cf *cf) {
    CFBins b;
    try {
        b = cf_bins_host(cf->nx, cf->ny);
    } catch (const std::invalid_argument &e) {
        throw Error(FR_EINVAL, e.what());
    }
    const int64_t J = (int64_t)b.k2.size();
    FR_REQUIRE(J >= 1, "grid too small for the amplitude model");
    cf->J = J;
    cf->t = DevBuf((size_t)J * 8);
    cf->d = DevBuf((size_t)J * 8);
    cf->mult = DevBuf((size_t)J * 8);
    cf->bin = DevBuf(b.bin.size() * 4);
    HIP_CHECK(hipMemcpy(cf->t.p, b.t.data(), cf->t.bytes, hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(cf->d.p, b.d.data(), cf->d.bytes, hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(cf->mult.p, b.mult.data(), cf->mult.bytes, hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(cf->bin.p, b.bin.data(), cf->bin.bytes, hipMemcpyHostToDevice));
}

size_t cf_scratch(const fr_cf *cf) { return scratch_round((size_t)(3 * cf->J + 1) * 8); }

template <typename T>
void cf_power(const fr_cf *cf, const double *prior, const double *xi_h, const double *xi_v, const double *xi_y,
              T *power, hipStream_t st) {
    CFPrior pr;
    for (int k = 0; k < 11; ++k) pr.v[k] = prior[k];
    const int64_t J = cf->J;
    Scratch work((size_t)(3 * J + 1) * 8, st);
    double *v = work.as<double>(), *logA = v + J, *P_bin = logA + J, *P0 = P_bin + J;
    k_cf_spectrum<<<1, kCFThreads, 0, st>>>(pr, J, (double)(cf->nx * cf->ny), cf->t.as<double>(),
                                            cf->d.as<double>(), cf->mult.as<double>(), xi_h, xi_v, xi_y, v, logA,
                                            P_bin, P0);
    LAUNCH_CHECK();
    map_async(CFScatter<T>{cf->bin.as<int32_t>(), P_bin, P0, power}, cf->nx * (cf->ny / 2 + 1), st);
}

// y[q] = offset + value (inverse row pass of the log-sky)
template <typename T> struct EpiAddConst {
    T *y;
    T offset;
    int ny;
    __device__ void operator()(int64_t row, int col, T v0, T v1) const {
        const int64_t q = row * ny + col;
        y[q] = offset + v0;
        y[q + 1] = offset + v1;
    }
};

// s = offset + F^-1 sqrt(P) F xi for n_img images of nx x ny
template <typename T>
void cf_logsky(const fr_cf *cf, const T *power, double offset, const T *xi, T *s, int64_t n_img, hipStream_t st) {
    const int64_t nx = cf->nx, ny = cf->ny;
    if (n_img == 0) return;
    ConvGeom g;
    g.n_img = n_img;
    g.rows_in = (int)nx;
    g.rows_out = (int)nx;
    g.n_in_cols = (int)ny;
    g.n_out_cols = (int)ny;
    g.log2M = ilog2(ny / 2);
    g.log2Lc = ilog2(nx);
    const Ctx &ctx = *cf->ctx;
    Scratch Y((size_t)n_img * nx * (ny / 2) * sizeof(c2<T>), st);
    launch_rfft_rows<T>(ctx, g, ProDiagScaled<T>{xi, nullptr, nullptr, (int)nx, (int)ny}, Y.as<c2<T>>(), st);
    launch_conv_cols<T>(ctx, g, Y.as<c2<T>>(), power, 1, 2 /* sqrt K */, T(1) / (T(nx) * T(ny / 2)), st);
    launch_irfft_rows<T>(ctx, g, EpiAddConst<T>{s, (T)offset, (int)ny}, Y.as<c2<T>>(), st);
}

template void cf_power<float>(const fr_cf *, const double *, const double *, const double *, const double *, float *,
                              hipStream_t);
template void cf_power<double>(const fr_cf *, const double *, const double *, const double *, const double *,
                               double *, hipStream_t);
template void cf_logsky<float>(const fr_cf *, const float *, double, const float *, float *, int64_t, hipStream_t);
template void cf_logsky<double>(const fr_cf *, const double *, double, const double *, double *, int64_t,
                                hipStream_t);

}  // namespace frmi
