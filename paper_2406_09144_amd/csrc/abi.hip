// extern "C" entry points of libfrmi: argument validation, precision dispatch,
// error translation.  All numerical work happens in the kernels of the other
// translation units.
#include <cmath>
#include <cstring>

#include "objects.h"
#include "profiler.h"

#include <atomic>
#include <mutex>

namespace frmi {

static thread_local std::string g_last_error;

void set_last_error(const std::string &m) { g_last_error = m; }

// allocations left before an injected failure (< 0: none injected)
static std::atomic<long long> g_alloc_budget{-1};

hipError_t device_alloc(void **p, size_t bytes) {
    long long b = g_alloc_budget.load();
    while (b >= 0) {
        if (b == 0) {
            *p = nullptr;
            g_alloc_budget.store(-1);  // one failure per injection
            return hipErrorOutOfMemory;
        }
        if (g_alloc_budget.compare_exchange_weak(b, b - 1)) break;
    }
    return hipMalloc(p, bytes);
}

// Workspace of fr_apply_RNR_approx_noalloc, for callers that cannot allocate:
// one copy per GPU, held until the process ends, shared by every such call on
// that GPU.  In host code `scratch` names a host-side stand-in, not device
// memory: kernels and copies get the device address found by
// hipGetSymbolAddress when a context is created on the device.
static __device__ __align__(256) unsigned char scratch[FR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kMaxDevices] = {};
static hipError_t g_noalloc_err[kMaxDevices] = {};
static bool g_noalloc_done[kMaxDevices] = {};

// Once per device, with that device current: the device address of `scratch`.
static void noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (g_noalloc_done[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_noalloc_err[device] = e;
    g_noalloc_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_noalloc_done[device] = true;
}

static void *noalloc_ptr(int device) {
    FR_REQUIRE(device >= 0 && device < kMaxDevices, "device index beyond the no-alloc workspace table");
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_done[device])
        throw Error(FR_EHIP, "no-alloc workspace: no context was created on this device");
    if (g_noalloc_err[device] != hipSuccess)
        throw Error(FR_EHIP, std::string("no-alloc workspace: hipGetSymbolAddress failed: ") +
                                 hipGetErrorString(g_noalloc_err[device]));
    return g_noalloc_ptr[device];
}

}  // namespace frmi

using namespace frmi;

#define FR_API_BEGIN try {
#define FR_API_END                                                 \
    }                                                              \
    catch (const frmi::Error &e) {                                 \
        set_last_error(e.what());                                  \
        return e.code;                                             \
    }                                                              \
    catch (const std::bad_alloc &) {                               \
        set_last_error("host allocation failed");                  \
        return FR_ENOMEM;                                          \
    }                                                              \
    catch (const std::exception &e) {                              \
        set_last_error(e.what());                                  \
        return FR_EHIP;                                            \
    }                                                              \
    set_last_error("");                                            \
    return FR_OK;

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

const char *fr_version(void) { return "frmi 0.1 (gfx950)"; }

const char *fr_last_error(void) { return g_last_error.c_str(); }

int fr_ctx_create(int device, fr_ctx **out) {
    FR_API_BEGIN
    FR_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_CHECK(hipGetDeviceCount(&ndev));
    FR_REQUIRE(device >= 0 && device < ndev, "device index out of range");
    DeviceGuard dg(device);
    auto ctx = std::make_unique<fr_ctx>();
    ctx->c.device = device;
    ctx->c.owner = ctx.get();
    HIP_CHECK(hipDeviceGetAttribute(&ctx->c.n_cu, hipDeviceAttributeMultiprocessorCount, device));
    // twiddle tables exp(-2 pi i m / L), computed in extended precision, rounded once
    auto make_table = [&](int64_t L, void **p64, void **p32) {
        std::vector<double> t64(2 * L);
        std::vector<float> t32(2 * L);
        for (int64_t m = 0; m < L; ++m) {
            long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)L;
            double c = (double)cosl(ang), s = (double)-sinl(ang);
            t64[2 * m] = c;
            t64[2 * m + 1] = s;
            t32[2 * m] = (float)c;
            t32[2 * m + 1] = (float)s;
        }
        DevBuf b64(t64.size() * sizeof(double)), b32(t32.size() * sizeof(float));
        HIP_CHECK(hipMemcpy(b64.p, t64.data(), b64.bytes, hipMemcpyHostToDevice));
        HIP_CHECK(hipMemcpy(b32.p, t32.data(), b32.bytes, hipMemcpyHostToDevice));
        *p64 = b64.p;
        *p32 = b32.p;
        ctx->tables.push_back(std::move(b64));
        ctx->tables.push_back(std::move(b32));
    };
    for (int l = 1; l <= kMaxLog2FFT + 1; ++l) make_table(int64_t(1) << l, &ctx->c.tw64[l], &ctx->c.tw32[l]);
    for (int o = 0; o < 2; ++o)
        for (int l = 0; l <= kMaxLog2Odd; ++l)
            make_table(int64_t(o == 0 ? 3 : 5) << l, &ctx->c.tw64o[o][l], &ctx->c.tw32o[o][l]);
    noalloc_setup(device);
    *out = ctx.release();
    FR_API_END
}

void fr_ctx_destroy(fr_ctx *ctx) {
    if (!ctx) return;
    try {
        DeviceGuard dg(ctx->c.device);
        delete ctx;
    } catch (...) {
        // the HIP runtime is already gone (process teardown): its memory goes with it
    }
}

static size_t real_size(bool fp64) { return fp64 ? 8 : 4; }

int fr_psf_create(fr_ctx *ctx, int64_t nx, int64_t ny, int64_t n_chan, const void *K_R, const void *K_N,
                  const void *nfac, int flags, fr_psf **out, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(ctx && out && K_R, "ctx, out and K_R are required");
    *out = nullptr;
    FR_REQUIRE(is_pow2(nx) && is_pow2(ny) && nx >= 16 && ny >= 16 && nx <= 8192 && ny <= 8192,
               "nx, ny must be powers of two in [16, 8192]");
    FR_REQUIRE(n_chan >= 1, "n_chan must be >= 1");
    FR_REQUIRE((flags & ~FR_FP64) == 0, "only FR_FP64 is a valid flag here");
    const bool fp64 = flags & FR_FP64;
    FR_REQUIRE(!fp64 || nx <= 4096, "FP64 PSF convolution supports nx <= 4096");
    DeviceGuard dg(ctx->c.device);
    hipStream_t st = as_stream(stream);
    auto p = std::make_unique<fr_psf>();
    p->ctx = &ctx->c;
    p->nx = nx;
    p->ny = ny;
    p->n_chan = n_chan;
    p->fp64 = fp64;
    p->px = 2 * nx;
    p->py = 2 * ny;
    const size_t rs = real_size(fp64);
    p->KR = DevBuf((size_t)n_chan * 2 * nx * (ny + 1) * rs);
    HIP_CHECK(hipMemcpyAsync(p->KR.p, K_R, p->KR.bytes, hipMemcpyDefault, st));
    if (K_N) {
        p->KN = DevBuf((size_t)n_chan * nx * (ny / 2 + 1) * rs);
        HIP_CHECK(hipMemcpyAsync(p->KN.p, K_N, p->KN.bytes, hipMemcpyDefault, st));
    }
    if (nfac) {
        p->nfac = DevBuf((size_t)nx * ny * rs);
        HIP_CHECK(hipMemcpyAsync(p->nfac.p, nfac, p->nfac.bytes, hipMemcpyDefault, st));
    }
    HIP_CHECK(hipStreamSynchronize(st));
    *out = p.release();
    FR_API_END
}

int fr_psf_get_kernels(const fr_psf *psf, void *K_R, void *K_N, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(psf, "psf is NULL");
    DeviceGuard dg(psf->ctx->device);
    hipStream_t st = as_stream(stream);
    if (K_R) HIP_CHECK(hipMemcpyAsync(K_R, psf->KR.p, psf->KR.bytes, hipMemcpyDefault, st));
    if (K_N) {
        FR_REQUIRE(psf->KN.p, "this PSF object has no noise kernel");
        HIP_CHECK(hipMemcpyAsync(K_N, psf->KN.p, psf->KN.bytes, hipMemcpyDefault, st));
    }
    FR_API_END
}

void fr_psf_destroy(fr_psf *psf) {
    if (!psf) return;
    try {
        DeviceGuard dg(psf->ctx->device);
        delete psf;
    } catch (...) {
        // the HIP runtime is already gone (process teardown): its memory goes with it
    }
}

int fr_apply_RNR_approx(fr_psf *psf, const void *x, void *y, int64_t B, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(psf, "psf is NULL");
    FR_REQUIRE(B >= 0, "B must be >= 0");
    if (B == 0) return FR_OK;
    FR_REQUIRE(x && y, "x and y are required");
    FR_REQUIRE(x != y, "y must not alias x");
    DeviceGuard dg(psf->ctx->device);
    if (psf->fp64)
        apply_rnr_approx<double>(psf, (const double *)x, (double *)y, B, as_stream(stream));
    else
        apply_rnr_approx<float>(psf, (const float *)x, (float *)y, B, as_stream(stream));
    FR_API_END
}

int fr_apply_RNR_approx_noalloc(fr_psf *psf, const void *x, void *y, int64_t B, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(psf, "psf is NULL");
    FR_REQUIRE(B >= 0, "B must be >= 0");
    if (B == 0) return FR_OK;
    FR_REQUIRE(x && y, "x and y are required");
    FR_REQUIRE(x != y, "y must not alias x");
    const size_t need = rnr_approx_scratch(psf, B);
    if (need > (size_t)FR_NOALLOC_SCRATCH_BYTES)
        throw Error(FR_EINVAL, "fr_apply_RNR_approx_noalloc: this call needs " + std::to_string(need) +
                                   " bytes of workspace, above the fixed " +
                                   std::to_string((size_t)FR_NOALLOC_SCRATCH_BYTES) +
                                   " (use fr_apply_RNR_approx or a smaller batch)");
    DeviceGuard dg(psf->ctx->device);
    void *ws = noalloc_ptr(psf->ctx->device);
    if (psf->fp64)
        apply_rnr_approx_ex<double>(psf, (const double *)x, nullptr, (double *)y, nullptr, nullptr, B,
                                    as_stream(stream), ws);
    else
        apply_rnr_approx_ex<float>(psf, (const float *)x, nullptr, (float *)y, nullptr, nullptr, B,
                                   as_stream(stream), ws);
    FR_API_END
}

int fr_fft2(fr_ctx *ctx, void *data, int64_t batch, int64_t n0, int64_t n1, int sign, int fp64, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(ctx && data, "ctx and data are required");
    FR_REQUIRE(batch >= 0, "batch must be >= 0");
    int o = 1, l = 0;
    FR_REQUIRE(split_len(n0, &o, &l) && split_len(n1, &o, &l) && n0 >= 2 && n1 >= 2 && n0 <= 16384 && n1 <= 16384,
               "sizes must be 2^p, 3 2^p or 5 2^p in [2, 16384]");
    FR_REQUIRE(!fp64 || (n0 <= 8192 && n1 <= 8192), "FP64 sizes are limited to 8192");
    FR_REQUIRE(sign == -1 || sign == 1, "sign must be -1 or +1");
    DeviceGuard dg(ctx->c.device);
    if (batch == 0) return FR_OK;
    if (fp64)
        fft2_inplace<double>(ctx->c, (double2 *)data, batch, n0, n1, sign, as_stream(stream));
    else
        fft2_inplace<float>(ctx->c, (float2 *)data, batch, n0, n1, sign, as_stream(stream));
    FR_API_END
}

int fr_plan_create(fr_ctx *ctx, const double *uvw_m, int64_t n_row, const double *freq_hz, int64_t n_chan,
                   int64_t nx, int64_t ny, double dx, double dy, double epsilon, int flags, int n_wplanes,
                   fr_plan **out) {
    FR_API_BEGIN
    FR_REQUIRE(ctx && out, "ctx and out are required");
    *out = nullptr;
    FR_REQUIRE(n_row >= 0 && n_chan >= 1, "n_row >= 0 and n_chan >= 1 required");
    FR_REQUIRE(n_row == 0 || uvw_m, "uvw_m is NULL");
    FR_REQUIRE(freq_hz, "freq_hz is NULL");
    FR_REQUIRE(is_pow2(nx) && is_pow2(ny) && nx >= 16 && ny >= 16 && nx <= 8192 && ny <= 8192,
               "nx, ny must be powers of two in [16, 8192]");
    FR_REQUIRE((flags & ~(FR_FP64 | FR_DIVIDE_BY_N | FR_COPLANAR | FR_W_TAYLOR | FR_VECTOR_SPREAD)) == 0,
               "unknown flag");
    const bool fp64 = flags & FR_FP64;
    FR_REQUIRE(!fp64 || (nx <= 4096 && ny <= 4096), "FP64 plans support nx, ny <= 4096");
    FR_REQUIRE(dx > 0 && dy > 0 && std::isfinite(dx) && std::isfinite(dy), "pixel sizes must be > 0");
    const double lm = (nx / 2) * dx, mm = (ny / 2) * dy;
    FR_REQUIRE(lm * lm + mm * mm < 1.0, "field of view must satisfy l^2 + m^2 < 1");
    FR_REQUIRE(epsilon >= 1e-14 && epsilon <= 1e-1, "epsilon must lie in [1e-14, 1e-1]");
    FR_REQUIRE(fp64 || epsilon >= 1e-6, "FP32 plans need epsilon >= 1e-6");
    FR_REQUIRE(n_wplanes >= 0, "n_wplanes must be >= 0");
    FR_REQUIRE(n_row * n_chan < (int64_t(1) << 31), "at most 2^31 - 1 visibilities per plan");
    for (int64_t c = 0; c < n_chan; ++c)
        FR_REQUIRE(freq_hz[c] > 0 && std::isfinite(freq_hz[c]), "frequencies must be > 0");
    for (int64_t r = 0; r < n_row; ++r)
        FR_REQUIRE(std::isfinite(uvw_m[3 * r]) && std::isfinite(uvw_m[3 * r + 1]) && std::isfinite(uvw_m[3 * r + 2]),
                   "uvw must be finite");
    DeviceGuard dg(ctx->c.device);
    auto pl = std::make_unique<fr_plan>();
    pl->ctx = &ctx->c;
    pl->nx = nx;
    pl->ny = ny;
    pl->nu = 2 * nx;
    pl->nv = 2 * ny;
    pl->n_row = n_row;
    pl->n_chan = n_chan;
    pl->n_vis = n_row * n_chan;
    pl->fp64 = fp64;
    pl->divide_by_n = flags & FR_DIVIDE_BY_N;
    pl->coplanar = flags & FR_COPLANAR;
    pl->want_taylor = flags & FR_W_TAYLOR;
    pl->vector_spread = flags & FR_VECTOR_SPREAD;
    pl->eps = epsilon;
    pl->dx_ = dx;
    pl->dy_ = dy;
    pl->n_wplanes_req = n_wplanes;
    pl->tile = 32;
    pl->freq.assign(freq_hz, freq_hz + n_chan);
    pl->uvw_host.assign(uvw_m, uvw_m + 3 * n_row);
    plan_build(pl.get(), uvw_m, freq_hz);
    *out = pl.release();
    FR_API_END
}

void fr_plan_destroy(fr_plan *plan) {
    if (!plan) return;
    try {
        DeviceGuard dg(plan->ctx->device);
        delete plan;
    } catch (...) {
        // the HIP runtime is already gone (process teardown): its memory goes with it
    }
}

int fr_plan_get_info(const fr_plan *pl, fr_plan_info *info) {
    FR_API_BEGIN
    FR_REQUIRE(pl && info, "plan and info are required");
    std::memset(info, 0, sizeof(*info));
    info->nx = pl->nx;
    info->ny = pl->ny;
    info->nu = pl->nu;
    info->nv = pl->nv;
    info->n_row = pl->n_row;
    info->n_chan = pl->n_chan;
    info->precision = pl->fp64 ? 64 : 32;
    info->support = pl->W;
    info->beta = pl->beta;
    info->coplanar = pl->coplanar ? 1 : 0;
    info->n_planes = pl->n_planes;
    info->w_support = pl->Ww;
    info->w_beta = pl->wbeta;
    info->w0 = pl->w0;
    info->dw = pl->dw;
    info->eps_bound = pl->eps_bound;
    info->tile = pl->tile;
    info->n_workitems = pl->n_wi;
    info->resident_bytes = pl->resident;
    info->w_taylor = pl->taylor ? 1 : 0;
    info->records_per_run = pl->vis_per_run;
    info->matrix_spread = frmi::matrix_spread(pl) ? 1 : 0;
    info->paired_degrid = frmi::paired_degrid(pl) ? 1 : 0;
    info->degrid_slots = pl->degrid_slots;
    info->active_tiles = pl->atile_chan.empty() ? 0 : pl->atile_chan.back();
    info->active_tile_cols = pl->tcol_chan.empty() ? 0 : pl->tcol_chan.back();
    FR_API_END
}

int fr_plan_export_order(const fr_plan *pl, uint64_t *keys, uint32_t *perm, int64_t *bucket_start,
                         int64_t *n_keys) {
    FR_API_BEGIN
    FR_REQUIRE(pl, "plan is NULL");
    DeviceGuard dg(pl->ctx->device);
    if (n_keys) *n_keys = plan_n_keys(pl);
    plan_export_order(pl, keys, perm, bucket_start);
    FR_API_END
}

int fr_degrid(fr_plan *pl, const void *img, void *vis, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(pl, "plan is NULL");
    if (pl->n_vis == 0) return FR_OK;
    FR_REQUIRE(img && vis, "img and vis are required");
    DeviceGuard dg(pl->ctx->device);
    if (pl->fp64)
        degrid<double>(pl, (const double *)img, (double2 *)vis, as_stream(stream));
    else
        degrid<float>(pl, (const float *)img, (float2 *)vis, as_stream(stream));
    FR_API_END
}

int fr_degrid_weighted(fr_plan *pl, const void *img, const void *weight, void *vis, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(pl, "plan is NULL");
    if (pl->n_vis == 0) return FR_OK;
    FR_REQUIRE(img && vis && weight, "img, weight and vis are required");
    DeviceGuard dg(pl->ctx->device);
    if (pl->fp64)
        degrid<double>(pl, (const double *)img, (double2 *)vis, as_stream(stream), (const double *)weight);
    else
        degrid<float>(pl, (const float *)img, (float2 *)vis, as_stream(stream), (const float *)weight);
    FR_API_END
}

int fr_grid(fr_plan *pl, const void *vis, const void *weight, void *img, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(pl, "plan is NULL");
    FR_REQUIRE(img, "img is required");
    FR_REQUIRE(pl->n_vis == 0 || vis, "vis is required");
    DeviceGuard dg(pl->ctx->device);
    if (pl->fp64)
        grid<double>(pl, (const double2 *)vis, (const double *)weight, (double *)img, as_stream(stream));
    else
        grid<float>(pl, (const float2 *)vis, (const float *)weight, (float *)img, as_stream(stream));
    FR_API_END
}

int fr_make_psf_kernel(fr_plan *pl, const void *weight, double eps_noise, fr_psf **out, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(pl && out, "plan and out are required");
    *out = nullptr;
    FR_REQUIRE(eps_noise != 0 && std::isfinite(eps_noise), "eps_noise must be non-zero and finite");
    FR_REQUIRE(pl->nx <= 4096 && pl->ny <= 4096, "PSF kernels need nx, ny <= 4096 (doubled grid)");
    FR_REQUIRE(!pl->fp64 || (pl->nx <= 2048 && pl->ny <= 2048), "FP64 PSF kernels need nx, ny <= 2048");
    DeviceGuard dg(pl->ctx->device);
    auto p = std::make_unique<fr_psf>();
    p->ctx = pl->ctx;
    p->nx = pl->nx;
    p->ny = pl->ny;
    p->n_chan = pl->n_chan;
    p->fp64 = pl->fp64;
    p->px = 2 * pl->nx;
    p->py = 2 * pl->ny;
    if (pl->fp64)
        make_psf<double>(pl, (const double *)weight, eps_noise, p.get(), as_stream(stream));
    else
        make_psf<float>(pl, (const float *)weight, eps_noise, p.get(), as_stream(stream));
    *out = p.release();
    FR_API_END
}

int fr_psf_reduce(const fr_psf *psf, int64_t hx, int64_t hy, fr_psf **out, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(psf && out, "psf and out are required");
    *out = nullptr;
    FR_REQUIRE(psf->px == 2 * psf->nx && psf->py == 2 * psf->ny, "psf must carry the full doubled-grid kernel");
    FR_REQUIRE(hx >= 0 && hx < psf->nx && hy >= 0 && hy < psf->ny, "support must satisfy 0 <= h < n per axis");
    DeviceGuard dg(psf->ctx->device);
    auto p = std::make_unique<fr_psf>();
    p->ctx = psf->ctx;
    p->nx = psf->nx;
    p->ny = psf->ny;
    p->n_chan = psf->n_chan;
    p->fp64 = psf->fp64;
    p->px = reduced_pad(psf->nx + hx);
    p->py = reduced_pad(psf->ny + hy);
    if (psf->fp64)
        reduce_psf<double>(psf, hx, hy, p.get(), as_stream(stream));
    else
        reduce_psf<float>(psf, hx, hy, p.get(), as_stream(stream));
    *out = p.release();
    FR_API_END
}

int fr_psf_get_padding(const fr_psf *psf, int64_t *px, int64_t *py) {
    FR_API_BEGIN
    FR_REQUIRE(psf && px && py, "psf, px and py are required");
    *px = psf->px;
    *py = psf->py;
    FR_API_END
}

int fr_apply_RNR_exact(fr_plan *pl, const void *weight, const void *x, void *y, int64_t B, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(pl, "plan is NULL");
    FR_REQUIRE(B >= 0, "B must be >= 0");
    if (B == 0) return FR_OK;
    FR_REQUIRE(x && y && x != y, "x and y are required and must differ");
    DeviceGuard dg(pl->ctx->device);
    if (pl->fp64)
        apply_rnr_exact<double>(pl, (const double *)weight, (const double *)x, (double *)y, B, as_stream(stream));
    else
        apply_rnr_exact<float>(pl, (const float *)weight, (const float *)x, (float *)y, B, as_stream(stream));
    FR_API_END
}

int fr_likelihood_grad(fr_plan *pl, fr_psf *psf, int mode, const void *s, const void *i_fixed, const void *data,
                       const void *weight, const void *inv_power, int64_t B, void *grad, double *H, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(mode == FR_LIK_EXACT || mode == FR_LIK_FAST, "mode must be FR_LIK_EXACT or FR_LIK_FAST");
    FR_REQUIRE(mode != FR_LIK_EXACT || pl, "FR_LIK_EXACT needs a plan");
    FR_REQUIRE(mode != FR_LIK_FAST || psf, "FR_LIK_FAST needs a PSF object");
    FR_REQUIRE(mode != FR_LIK_FAST || psf->KN.p, "FR_LIK_FAST needs a PSF object with a noise kernel");
    FR_REQUIRE(B >= 0, "B must be >= 0");
    if (B == 0) return FR_OK;
    FR_REQUIRE(s && data && grad && H, "s, data, grad and H are required");
    const bool fp64 = mode == FR_LIK_FAST ? psf->fp64 : pl->fp64;
    DeviceGuard dg(mode == FR_LIK_FAST ? psf->ctx->device : pl->ctx->device);
    if (fp64)
        likelihood_grad<double>(pl, psf, mode, (const double *)s, (const double *)i_fixed, data,
                                (const double *)weight, (const double *)inv_power, B, (double *)grad, H,
                                as_stream(stream));
    else
        likelihood_grad<float>(pl, psf, mode, (const float *)s, (const float *)i_fixed, data, (const float *)weight,
                               (const float *)inv_power, B, (float *)grad, H, as_stream(stream));
    FR_API_END
}

int fr_cg_solve(fr_plan *pl, fr_psf *psf, const void *weight, const void *inv_power, const void *diag,
                const void *b, void *x, int maxiter, double rtol, double *resid_hist, int *iters_done, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(pl || psf, "a plan or a PSF object is required");
    FR_REQUIRE(b && x && resid_hist && iters_done, "b, x, resid_hist and iters_done are required");
    FR_REQUIRE(b != x, "x must not alias b");
    FR_REQUIRE(maxiter >= 0 && rtol >= 0 && std::isfinite(rtol), "maxiter >= 0 and rtol >= 0 required");
    const bool fp64 = psf ? psf->fp64 : pl->fp64;
    if (psf && pl)
        FR_REQUIRE(pl->nx == psf->nx && pl->ny == psf->ny && pl->n_chan == psf->n_chan && pl->fp64 == psf->fp64,
                   "plan and PSF object disagree on shape or precision");
    DeviceGuard dg(psf ? psf->ctx->device : pl->ctx->device);
    if (fp64)
        cg_solve<double>(pl, psf, (const double *)weight, (const double *)inv_power, (const double *)diag,
                         (const double *)b, (double *)x, maxiter, rtol, resid_hist, iters_done, as_stream(stream));
    else
        cg_solve<float>(pl, psf, (const float *)weight, (const float *)inv_power, (const float *)diag,
                        (const float *)b, (float *)x, maxiter, rtol, resid_hist, iters_done, as_stream(stream));
    FR_API_END
}

int fr_periodic_conv(fr_ctx *ctx, const void *K, int64_t nk, int mode, const void *x, void *y, int64_t n_img,
                     int64_t nx, int64_t ny, int fp64, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(ctx && K, "ctx and K are required");
    FR_REQUIRE(n_img >= 0 && nk >= 1, "n_img >= 0 and nk >= 1 required");
    FR_REQUIRE(mode >= FR_CONV_MUL && mode <= FR_CONV_DIV_SQRT, "unknown mode");
    FR_REQUIRE(is_pow2(nx) && is_pow2(ny) && nx >= 4 && ny >= 4 && nx <= 8192 && ny <= 8192,
               "nx, ny must be powers of two in [4, 8192]");
    FR_REQUIRE(!fp64 || (nx <= 4096 && ny <= 8192), "FP64 periodic convolutions need nx <= 4096");
    if (n_img == 0) return FR_OK;
    FR_REQUIRE(x && y && x != y, "x and y are required and must differ");
    DeviceGuard dg(ctx->c.device);
    if (fp64)
        periodic_conv_ex<double>(ctx->c, (const double *)x, nullptr, (double *)y, nullptr, nullptr, n_img, nx, ny,
                                 (const double *)K, (int)nk, mode, as_stream(stream));
    else
        periodic_conv_ex<float>(ctx->c, (const float *)x, nullptr, (float *)y, nullptr, nullptr, n_img, nx, ny,
                                (const float *)K, (int)nk, mode, as_stream(stream));
    FR_API_END
}

int fr_cf_create(fr_ctx *ctx, int64_t nx, int64_t ny, fr_cf **out) {
    FR_API_BEGIN
    FR_REQUIRE(ctx && out, "ctx and out are required");
    *out = nullptr;
    FR_REQUIRE(is_pow2(nx) && is_pow2(ny) && nx >= 4 && ny >= 4 && nx <= 8192 && ny <= 8192,
               "nx, ny must be powers of two in [4, 8192]");
    DeviceGuard dg(ctx->c.device);
    auto cf = std::make_unique<fr_cf>();
    cf->ctx = &ctx->c;
    cf->nx = nx;
    cf->ny = ny;
    cf_build(cf.get());
    *out = cf.release();
    FR_API_END
}

int fr_cf_num_bins(const fr_cf *cf, int64_t *n_bins) {
    FR_API_BEGIN
    FR_REQUIRE(cf && n_bins, "cf and n_bins are required");
    *n_bins = cf->J;
    FR_API_END
}

void fr_cf_destroy(fr_cf *cf) {
    if (!cf) return;
    try {
        DeviceGuard dg(cf->ctx->device);
        delete cf;
    } catch (...) {
        // the HIP runtime is already gone (process teardown): its memory goes with it
    }
}

int fr_cf_power(fr_cf *cf, const double *prior, const double *xi_hyper, const double *xi_v, const double *xi_y,
                void *power, int fp64, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(cf && prior && xi_hyper && xi_v && xi_y && power, "every argument is required");
    for (int k : {1, 3, 7, 9}) {
        FR_REQUIRE(std::isfinite(prior[k]) && prior[k] >= 0.0, "lognormal means must be >= 0");
        FR_REQUIRE(std::isfinite(prior[k + 1]) && prior[k + 1] >= 0.0, "standard deviations must be >= 0");
    }
    FR_REQUIRE(prior[1] > 0.0 && prior[3] > 0.0, "zero-mode std and fluctuations means must be > 0");
    FR_REQUIRE(std::isfinite(prior[0]) && std::isfinite(prior[5]) && std::isfinite(prior[6]) && prior[6] >= 0.0,
               "offset and slope must be finite, slope std >= 0");
    DeviceGuard dg(cf->ctx->device);
    if (fp64)
        cf_power<double>(cf, prior, xi_hyper, xi_v, xi_y, (double *)power, as_stream(stream));
    else
        cf_power<float>(cf, prior, xi_hyper, xi_v, xi_y, (float *)power, as_stream(stream));
    FR_API_END
}

int fr_cf_logsky(fr_cf *cf, const void *power, double offset, const void *xi, void *s, int64_t n_img, int fp64,
                 void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(cf && power, "cf and power are required");
    FR_REQUIRE(n_img >= 0, "n_img must be >= 0");
    FR_REQUIRE(std::isfinite(offset), "offset must be finite");
    if (n_img == 0) return FR_OK;
    FR_REQUIRE(xi && s && xi != s, "xi and s are required and must differ");
    FR_REQUIRE(!fp64 || cf->nx <= 4096, "FP64 needs nx <= 4096");
    DeviceGuard dg(cf->ctx->device);
    if (fp64)
        cf_logsky<double>(cf, (const double *)power, offset, (const double *)xi, (double *)s, n_img,
                          as_stream(stream));
    else
        cf_logsky<float>(cf, (const float *)power, offset, (const float *)xi, (float *)s, n_img, as_stream(stream));
    FR_API_END
}

static void mgvi_check(const fr_psf *psf, const void *power) {
    FR_REQUIRE(psf && power, "psf and power are required");
    FR_REQUIRE(psf->KN.p, "the PSF object has no noise kernel (N'^-1 is part of the metric)");
}

int fr_mgvi_metric_apply(fr_psf *psf, const void *power, const void *diag, const void *x, void *y, void *stream) {
    FR_API_BEGIN
    mgvi_check(psf, power);
    FR_REQUIRE(x && y && x != y, "x and y are required and must differ");
    DeviceGuard dg(psf->ctx->device);
    if (psf->fp64)
        mgvi_metric_apply<double>(psf, (const double *)power, (const double *)diag, (const double *)x, (double *)y,
                                  as_stream(stream));
    else
        mgvi_metric_apply<float>(psf, (const float *)power, (const float *)diag, (const float *)x, (float *)y,
                                 as_stream(stream));
    FR_API_END
}

int fr_mgvi_draw(fr_psf *psf, const void *power, const void *diag, const void *eta0, const void *eta1, void *xi,
                 void *stream) {
    FR_API_BEGIN
    mgvi_check(psf, power);
    FR_REQUIRE(eta0 && eta1 && xi, "eta0, eta1 and xi are required");
    FR_REQUIRE(xi != eta0 && xi != eta1, "xi must not alias eta0 or eta1");
    DeviceGuard dg(psf->ctx->device);
    if (psf->fp64)
        mgvi_draw<double>(psf, (const double *)power, (const double *)diag, (const double *)eta0,
                          (const double *)eta1, (double *)xi, as_stream(stream));
    else
        mgvi_draw<float>(psf, (const float *)power, (const float *)diag, (const float *)eta0, (const float *)eta1,
                         (float *)xi, as_stream(stream));
    FR_API_END
}

int fr_mgvi_solve(fr_psf *psf, const void *power, const void *diag, const void *b, void *x, int maxiter, double rtol,
                  double *resid_hist, int *iters_done, void *stream) {
    FR_API_BEGIN
    mgvi_check(psf, power);
    FR_REQUIRE(b && x && resid_hist && iters_done, "b, x, resid_hist and iters_done are required");
    FR_REQUIRE(b != x, "x must not alias b");
    FR_REQUIRE(maxiter >= 0 && rtol >= 0 && std::isfinite(rtol), "maxiter >= 0 and rtol >= 0 required");
    DeviceGuard dg(psf->ctx->device);
    if (psf->fp64)
        mgvi_solve<double>(psf, (const double *)power, (const double *)diag, (const double *)b, (double *)x, maxiter,
                           rtol, resid_hist, iters_done, as_stream(stream));
    else
        mgvi_solve<float>(psf, (const float *)power, (const float *)diag, (const float *)b, (float *)x, maxiter, rtol,
                          resid_hist, iters_done, as_stream(stream));
    FR_API_END
}

int fr_query_footprint(const fr_plan *pl, const fr_psf *psf, int op, int64_t B, size_t *scratch_bytes,
                       size_t *resident_bytes) {
    FR_API_BEGIN
    FR_REQUIRE(scratch_bytes && resident_bytes, "outputs are required");
    FR_REQUIRE(B >= 0, "B must be >= 0");
    FR_REQUIRE(op >= FR_OP_DEGRID && op <= FR_OP_MAKE_PSF, "unknown op");
    const bool need_plan = op == FR_OP_DEGRID || op == FR_OP_GRID || op == FR_OP_RNR_EXACT ||
                           op == FR_OP_LIK_EXACT || op == FR_OP_MAKE_PSF;
    FR_REQUIRE(!need_plan || pl, "this op needs a plan");
    FR_REQUIRE(need_plan || op == FR_OP_CG || psf, "this op needs a PSF object");
    FR_REQUIRE(op != FR_OP_CG || pl || psf, "CG needs a plan or a PSF object");
    const bool prior = true;  // the prior term's scratch is counted whenever an op can take one
    size_t s = 0;
    switch (op) {
    case FR_OP_DEGRID: s = pl->n_vis ? degrid_scratch(pl) : 0; break;
    case FR_OP_GRID: s = grid_scratch(pl); break;
    case FR_OP_RNR_APPROX: s = rnr_approx_scratch(psf, B); break;
    case FR_OP_RNR_EXACT: s = B ? rnr_exact_scratch(pl) : 0; break;
    case FR_OP_LIK_FAST: s = B ? lik_scratch(pl, psf, FR_LIK_FAST, B, prior) : 0; break;
    case FR_OP_LIK_EXACT: s = B ? lik_scratch(pl, psf, FR_LIK_EXACT, B, prior) : 0; break;
    case FR_OP_CG: s = cg_scratch(pl, psf, prior); break;
    case FR_OP_MAKE_PSF: s = psf_build_scratch(pl) + psf_plan_device_bound(pl); break;
    }
    *scratch_bytes = s;
    size_t r = 0;
    if (pl) r += pl->resident;
    if (psf) r += psf->KR.bytes + psf->KN.bytes + psf->nfac.bytes;
    *resident_bytes = r;
    FR_API_END
}

int fr_scratch_stats(fr_ctx *ctx, void *stream, int reset, size_t *peak_in_use, size_t *held) {
    FR_API_BEGIN
    FR_REQUIRE(ctx && peak_in_use && held, "ctx, peak_in_use and held are required");
    DeviceGuard dg(ctx->c.device);
    Arena &a = arena_for(as_stream(stream));
    *held = a.held();
    *peak_in_use = a.peak(reset != 0);
    FR_API_END
}

int fr_scratch_trim(fr_ctx *ctx, void *stream) {
    FR_API_BEGIN
    FR_REQUIRE(ctx, "ctx is NULL");
    DeviceGuard dg(ctx->c.device);
    HIP_CHECK(hipStreamSynchronize(as_stream(stream)));
    if (!arena_for(as_stream(stream)).trim()) throw Error(FR_EBUSY, "scratch of this stream is in use");
    FR_API_END
}

int fr_inject_alloc_failure(int64_t after) {
    FR_API_BEGIN
    FR_REQUIRE(after >= -1, "after must be >= -1");
    g_alloc_budget.store(after);
    FR_API_END
}

}  // extern "C"

namespace frmi {
Profiler &profiler() {
    static Profiler P;
    return P;
}

Arena &arena_for(hipStream_t st) {
    static std::mutex mu;
    // never destroyed: the runtime may be gone when static destructors run
    static auto *arenas = new std::map<std::pair<int, hipStream_t>, std::unique_ptr<Arena>>();
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto &slot = (*arenas)[{dev, st}];
    if (!slot) slot = std::make_unique<Arena>();
    return *slot;
}
}  // namespace frmi

extern "C" {

int fr_profile_enable(int on) {
    FR_API_BEGIN
    Profiler &P = profiler();
    std::lock_guard<std::mutex> g(P.mu);
    P.on = on != 0;
    // create the events up front so that timed regions only record them
    while (P.on && P.pool.size() < kProfilerPoolEvents) {
        hipEvent_t e;
        HIP_CHECK(hipEventCreate(&e));
        P.pool.push_back(e);
    }
    FR_API_END
}

int fr_profile_reset(void) {
    FR_API_BEGIN
    Profiler &P = profiler();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto &kv : P.recs)
        for (auto &r : kv.second) {
            (void)hipEventSynchronize(r.b);
            P.pool.push_back(r.a);
            P.pool.push_back(r.b);
        }
    P.recs.clear();
    FR_API_END
}

int fr_profile_query(const char *name, int64_t *launches, double *total_ms) {
    FR_API_BEGIN
    FR_REQUIRE(name && launches && total_ms, "name, launches and total_ms are required");
    Profiler &P = profiler();
    std::lock_guard<std::mutex> g(P.mu);
    *launches = 0;
    *total_ms = 0;
    auto it = P.recs.find(name);
    if (it == P.recs.end()) return FR_OK;
    for (auto &r : it->second) {
        HIP_CHECK(hipEventSynchronize(r.b));
        float ms = 0;
        HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
        *total_ms += ms;
        *launches += 1;
    }
    FR_API_END
}

}  // extern "C"
