// Response and noise kernels of the PSF approximation (Sec. 3.3.2, Sec. 3.3.3),
// computed on the GPU from the plan's visibilities and weights.
//
//   PSF0 = R0^+ N^-1 R0 delta on the 2nx x 2ny grid: gridding the weights (all
//          visibilities = 1) with a coplanar plan of the doubled image, no 1/n;
//   K_R  = Re fft2(ifftshift(PSF0)) with the offset -nx row / -ny column zeroed
//          (they never enter the cropped linear convolution, and without them
//          PSF0 is periodically even so K_R is real), kept on the r2c half;
//   K_N  = eps + max(Re fft2(ifftshift(crop PSF0)), 0), crop = offsets [-n/2, n/2):
//          the per-frequency minimiser of the squared residual between N' and
//          the kernel convolution on a central point source (closed form of the
//          argmin over xi; where Re T <= 0 the infimum exp(xi) -> 0 gives eps).
#include <algorithm>
#include <climits>

#include "elementwise.h"
#include "objects.h"

namespace frmi {

template <typename T> struct ShiftPsfFull {
    const T *psf;  // [nc][2nx][2ny]
    c2<T> *z;      // [nc][2nx][2ny]
    int64_t nx, ny;
    __device__ void operator()(int64_t q) const {
        const int64_t n2x = 2 * nx, n2y = 2 * ny;
        const int64_t c = q / (n2x * n2y);
        const int64_t r = q - c * n2x * n2y;
        const int64_t i = r / n2y, j = r - i * n2y;
        const int64_t si = (i + nx) & (n2x - 1), sj = (j + ny) & (n2y - 1);
        const T v = (si == 0 || sj == 0) ? T(0) : psf[(c * n2x + si) * n2y + sj];
        z[q] = mk<T>(v, T(0));
    }
};

template <typename T> struct ExtractKR {
    const c2<T> *z;  // [nc][2nx][2ny]
    T *kr;           // [nc][2nx][ny + 1]
    int64_t nx, ny;
    __device__ void operator()(int64_t q) const {
        const int64_t w = ny + 1;
        const int64_t row = q / w, j = q - row * w;  // row = c * 2nx + i
        kr[q] = z[row * 2 * ny + j].x;
    }
};

template <typename T> struct ShiftPsfCrop {
    const T *psf;  // [nc][2nx][2ny]
    c2<T> *z;      // [nc][nx][ny]
    int64_t nx, ny;
    __device__ void operator()(int64_t q) const {
        const int64_t c = q / (nx * ny);
        const int64_t r = q - c * nx * ny;
        const int64_t i = r / ny, j = r - i * ny;
        const int64_t oi = i < nx / 2 ? i : i - nx;  // offset held by index i after ifftshift
        const int64_t oj = j < ny / 2 ? j : j - ny;
        z[q] = mk<T>(psf[(c * 2 * nx + nx + oi) * 2 * ny + ny + oj], T(0));
    }
};

template <typename T> struct ExtractKN {
    const c2<T> *z;  // [nc][nx][ny]
    const T *psf;    // [nc][2nx][2ny], for the relative regulariser
    T *kn;           // [nc][nx][ny/2 + 1]
    int64_t nx, ny;
    double eps;      // > 0 absolute, < 0 relative to the PSF peak
    __device__ void operator()(int64_t q) const {
        const int64_t w = ny / 2 + 1;
        const int64_t row = q / w, j = q - row * w;
        const int64_t c = row / nx;
        T e = (T)eps;
        if (eps < 0) e = (T)(-eps) * psf[(c * 2 * nx + nx) * 2 * ny + ny];
        const T t = z[row * ny + j].x;
        kn[q] = e + (t > T(0) ? t : T(0));
    }
};

size_t psf_build_scratch(const fr_plan *pl) {
    const size_t rs = pl->fp64 ? 8 : 4;
    const size_t n_psf = (size_t)pl->n_chan * 4 * pl->nx * pl->ny;
    return scratch_round(n_psf * rs) + std::max(psf_grid_scratch_bound(pl), scratch_round(n_psf * 2 * rs));
}

template <typename T>
void make_psf(fr_plan *pl, const T *weight, double eps_noise, fr_psf *out, hipStream_t st) {
    const int64_t nx = pl->nx, ny = pl->ny, nc = pl->n_chan;
    // coplanar plan of the doubled field, same pixel size, no 1/n
    fr_plan *sp = nullptr;
    const int flags = FR_COPLANAR | (pl->fp64 ? FR_FP64 : 0);
    const int rc = fr_plan_create((fr_ctx *)pl->ctx->owner, pl->uvw_host.data(), pl->n_row, pl->freq.data(), nc,
                                  2 * nx, 2 * ny, pl->dx_, pl->dy_, pl->eps, flags, 0, &sp);
    if (rc != FR_OK) throw Error(rc, std::string("PSF plan: ") + fr_last_error());
    // kernels in flight read the sub-plan: make sure they are done before it goes
    auto release = [st](fr_plan *p) {
        (void)hipStreamSynchronize(st);
        fr_plan_destroy(p);
    };
    std::unique_ptr<fr_plan, decltype(release)> guard(sp, release);
    const int64_t n_psf = nc * 4 * nx * ny;
    Scratch psf0(n_psf * sizeof(T), st);
    grid<T>(sp, nullptr, weight, psf0.as<T>(), st);
    Scratch z(n_psf * sizeof(c2<T>), st);
    map_async(ShiftPsfFull<T>{psf0.as<T>(), z.as<c2<T>>(), nx, ny}, n_psf, st);
    fft2_inplace<T>(*pl->ctx, z.as<c2<T>>(), nc, 2 * nx, 2 * ny, -1, st);
    out->KR = DevBuf((size_t)nc * 2 * nx * (ny + 1) * sizeof(T));
    map_async(ExtractKR<T>{z.as<c2<T>>(), out->KR.as<T>(), nx, ny}, nc * 2 * nx * (ny + 1), st);
    map_async(ShiftPsfCrop<T>{psf0.as<T>(), z.as<c2<T>>(), nx, ny}, nc * nx * ny, st);
    fft2_inplace<T>(*pl->ctx, z.as<c2<T>>(), nc, nx, ny, -1, st);
    out->KN = DevBuf((size_t)nc * nx * (ny / 2 + 1) * sizeof(T));
    map_async(ExtractKN<T>{z.as<c2<T>>(), psf0.as<T>(), out->KN.as<T>(), nx, ny, eps_noise}, nc * nx * (ny / 2 + 1),
              st);
    if (pl->divide_by_n) {
        out->nfac = DevBuf(pl->nfac.bytes);
        HIP_CHECK(hipMemcpyAsync(out->nfac.p, pl->nfac.p, pl->nfac.bytes, hipMemcpyDeviceToDevice, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------- reduced support
// Sec. 3.3.2: neglecting the PSF sidelobes beyond |offset| > h lets the zero
// padding shrink from 2n to n + h per axis (the smallest FFT length of the form
// 2^p, 3 2^p or 5 2^p that is even and >= n + h), with no wrapped term reaching
// the cropped window.
int64_t reduced_pad(int64_t n) {
    int64_t best = 0;
    for (int64_t odd : {1, 3, 5}) {
        int64_t m = 2 * odd;
        while (m < n) m *= 2;
        if (best == 0 || m < best) best = m;
    }
    return best;
}

// Full real spectrum [nc][2nx][2ny] from the r2c half of an even kernel: K[-k] = K[k].
template <typename T> struct ExpandKR {
    const T *kr;  // [nc][2nx][ny + 1]
    c2<T> *z;     // [nc][2nx][2ny]
    int64_t nx, ny;
    __device__ void operator()(int64_t q) const {
        const int64_t n2x = 2 * nx, n2y = 2 * ny;
        const int64_t c = q / (n2x * n2y);
        const int64_t r = q - c * n2x * n2y;
        const int64_t i = r / n2y, j = r - i * n2y;
        const int64_t si = j <= ny ? i : (n2x - i) & (n2x - 1), sj = j <= ny ? j : n2y - j;
        z[q] = mk<T>(kr[(c * n2x + si) * (ny + 1) + sj], T(0));
    }
};

// The PSF (periodic layout on the doubled grid, scaled by 4 nx ny after the inverse
// FFT) restricted to |dx| <= hx, |dy| <= hy and placed on the px x py grid.
template <typename T> struct PlaceTruncated {
    const c2<T> *z;  // [nc][2nx][2ny]
    c2<T> *out;      // [nc][px][py]
    int64_t nx, ny, px, py, hx, hy;
    T inv;           // 1 / (4 nx ny)
    __device__ void operator()(int64_t q) const {
        const int64_t c = q / (px * py);
        const int64_t r = q - c * px * py;
        const int64_t a = r / py, b = r - a * py;
        const int64_t dx = a <= hx ? a : (a >= px - hx ? a - px : INT64_MAX);
        const int64_t dy = b <= hy ? b : (b >= py - hy ? b - py : INT64_MAX);
        T v = T(0);
        if (dx != INT64_MAX && dy != INT64_MAX)
            v = z[(c * 2 * nx + (dx & (2 * nx - 1))) * 2 * ny + (dy & (2 * ny - 1))].x * inv;
        out[q] = mk<T>(v, T(0));
    }
};

template <typename T> struct ExtractKRed {
    const c2<T> *z;  // [nc][px][py]
    T *kr;           // [nc][px][py/2 + 1]
    int64_t py;
    __device__ void operator()(int64_t q) const {
        const int64_t w = py / 2 + 1;
        const int64_t row = q / w, j = q - row * w;
        kr[q] = z[row * py + j].x;
    }
};

template <typename T>
void reduce_psf(const fr_psf *in, int64_t hx, int64_t hy, fr_psf *out, hipStream_t st) {
    const int64_t nx = in->nx, ny = in->ny, nc = in->n_chan, px = out->px, py = out->py;
    const Ctx &ctx = *in->ctx;
    const int64_t n_full = nc * 4 * nx * ny, n_red = nc * px * py;
    Scratch z(n_full * sizeof(c2<T>), st);
    map_async(ExpandKR<T>{in->KR.as<T>(), z.as<c2<T>>(), nx, ny}, n_full, st);
    fft2_inplace<T>(ctx, z.as<c2<T>>(), nc, 2 * nx, 2 * ny, +1, st);
    Scratch zr(n_red * sizeof(c2<T>), st);
    map_async(PlaceTruncated<T>{z.as<c2<T>>(), zr.as<c2<T>>(), nx, ny, px, py, hx, hy, T(1) / (T(4 * nx) * T(ny))},
              n_red, st);
    fft2_inplace<T>(ctx, zr.as<c2<T>>(), nc, px, py, -1, st);
    out->KR = DevBuf((size_t)nc * px * (py / 2 + 1) * sizeof(T));
    map_async(ExtractKRed<T>{zr.as<c2<T>>(), out->KR.as<T>(), py}, nc * px * (py / 2 + 1), st);
    if (in->KN.p) {
        out->KN = DevBuf(in->KN.bytes);
        HIP_CHECK(hipMemcpyAsync(out->KN.p, in->KN.p, in->KN.bytes, hipMemcpyDeviceToDevice, st));
    }
    if (in->nfac.p) {
        out->nfac = DevBuf(in->nfac.bytes);
        HIP_CHECK(hipMemcpyAsync(out->nfac.p, in->nfac.p, in->nfac.bytes, hipMemcpyDeviceToDevice, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
}

template void reduce_psf<float>(const fr_psf *, int64_t, int64_t, fr_psf *, hipStream_t);
template void reduce_psf<double>(const fr_psf *, int64_t, int64_t, fr_psf *, hipStream_t);

template void make_psf<float>(fr_plan *, const float *, double, fr_psf *, hipStream_t);
template void make_psf<double>(fr_plan *, const double *, double, fr_psf *, hipStream_t);

}  // namespace frmi
