// Opaque objects behind the C ABI and the internal entry points between
// translation units.
#pragma once

#include "common.h"
#include "workitem.h"

struct fr_ctx {
    frmi::Ctx c;
    std::vector<frmi::DevBuf> tables;
};

// Per-channel response and noise kernels of the PSF approximation (Sec. 3.3.2-3.3.3).
struct fr_psf {
    frmi::Ctx *ctx = nullptr;
    int64_t nx = 0, ny = 0, n_chan = 0;
    bool fp64 = false;
    int64_t px = 0, py = 0;  // periodic grid of the response kernel: 2nx x 2ny, smaller when reduced
    frmi::DevBuf KR;    // [n_chan][px][py/2 + 1] real
    frmi::DevBuf KN;    // [n_chan][nx][ny/2 + 1] real (empty if absent)
    frmi::DevBuf nfac;  // [nx][ny] real diagonal D (empty = identity)
};


// Correlated-field amplitude model on an nx x ny grid: the distinct non-zero |k|
// (bins), their log-frequencies and steps, multiplicities, and the bin of every
// r2c half-spectrum cell.
struct fr_cf {
    frmi::Ctx *ctx = nullptr;
    int64_t nx = 0, ny = 0, J = 0;
    frmi::DevBuf t, d, mult;  // double [J]
    frmi::DevBuf bin;         // int32 [nx][ny/2 + 1], -1 at k = 0
};

struct fr_plan {
    frmi::Ctx *ctx = nullptr;
    int64_t nx = 0, ny = 0, nu = 0, nv = 0, n_row = 0, n_chan = 0;
    bool fp64 = false, divide_by_n = false, coplanar = true;
    int W = 0;          // uv kernel support (cells)
    double beta = 0;    // uv kernel shape
    int Ww = 1;         // w kernel support (planes)
    double wbeta = 0;
    double w_xmax = 0.25;  // bound of the w-image coordinate dw |t| the kernel was chosen for
    int n_planes = 1;
    double w0 = 0, dw = 1, yc = 0;  // plane p at w0 + p dw; n - 1 measured from yc
    bool want_taylor = false;       // FR_W_TAYLOR requested
    bool vector_spread = false;     // FR_VECTOR_SPREAD: never the matrix-core spread
    bool taylor = false;            // planes are the Taylor terms of exp(-2 pi i w t)
    double taylor_h = 0;            // |t| <= h over the image
    int tile = 32;
    double eps = 0, eps_bound = 0;
    double dx_ = 0, dy_ = 0;  // pixel sizes (radians)
    int n_wplanes_req = 0;
    int64_t n_vis = 0;
    int64_t max_wi_count = 0;
    // per-pixel factors (precision of the plan)
    frmi::DevBuf fac;   // [nx][ny] a / (Psi_u Psi_v Psi_w)
    frmi::DevBuf tpix;    // [nx][ny] ((n - 1) - yc) / h (Taylor plans only, plan precision)
    frmi::DevBuf tpix_w;  // [nx][ny] double (n - 1) - yc (w-stacked plans only)
    frmi::DevBuf nfac;  // [nx][ny] a (1/n or 1)
    frmi::DevBuf wplane;  // [n_planes] double: w of each plane
    // sorted visibility records (structure of arrays)
    frmi::DevBuf r_idx;   // uint32 [n_vis]: row * n_chan + chan, bit 31 = conjugate
    frmi::DevBuf r_pos;   // uint32 [n_vis]: record position of visibility row * n_chan + chan, bit 31 = conjugate
    frmi::DevBuf dpair;   // uint32 [n_vis] (paired degridding): pair list of each degridding item from its start
    frmi::DevBuf r_cell;  // uint32 [n_vis]: (a0 - tu) | (b0 - tv) << 16
    frmi::DevBuf r_du, r_dv, r_dw, r_ph;  // T [n_vis]
    frmi::DevBuf wi;      // WorkItem [n_wi]
    int64_t n_wi = 0;
    std::vector<int64_t> wi_chan;  // work-item range per channel, [n_chan + 1]
    // gridding items: pieces of one key each, and per key the first item; the
    // items of a channel are split into consecutive ranges of about equal
    // estimated cost, one per workgroup of the spread
    frmi::DevBuf gwi;        // WorkItem [n_gwi]
    frmi::DevBuf gseg;       // int32, per channel: first item of each workgroup (from the
                             // channel's first item), then the channel's item count
    std::vector<int64_t> gseg_chan;  // [n_chan + 1] offsets of each channel's block in gseg
    double vis_per_run = 0;  // records per run of equal (bucket, base cell)
    int64_t degrid_slots = 0;  // pair-list entries (paired degridding) or records
    int64_t n_gwi = 0;
    std::vector<int64_t> gwi_chan;
    frmi::DevBuf gkey_first;  // uint32 [n_keys + 1]
    // tiles whose planes can be non-zero (an item of the tile, or of the tile one
    // step back in u and/or v, whose halo reaches in): a list per channel and a
    // per-channel map that lets the inverse column FFT skip the others
    frmi::DevBuf atile;                 // int32 tile index [sum over channels]
    std::vector<int64_t> atile_chan;    // [n_chan + 1] offsets into atile
    frmi::DevBuf tile_active;           // uint8 [n_chan][n_tiles]
    // tile columns (kTile grid columns each) holding an active tile: a map per
    // channel, and per channel the list of them, so that the w-plane column
    // transforms and the row passes leave the others alone
    frmi::DevBuf col_active;            // uint8 [n_chan][ntv]
    frmi::DevBuf tcol;                  // int32 active tile columns of each channel, ascending
    std::vector<int64_t> tcol_chan;     // [n_chan + 1] offsets into tcol
    int n_p0 = 1, n_tiles = 1, ntu = 1, ntv = 1;
    std::vector<double> freq;
    std::vector<double> uvw_host;  // [n_row][3] metres, kept to derive the PSF plan
    size_t resident = 0;
};

namespace frmi {

// FP32 gridding of plans with W <= 8 runs the spread on the matrix cores when the
// sorted records average at least 4 per run of equal base cell (one MFMA step
// takes four records of a run); otherwise it stays on the vector units.
inline bool matrix_spread(const fr_plan *pl) {
    return !pl->fp64 && !pl->vector_spread && pl->W <= 8 && pl->vis_per_run >= 4.0;
}
// degridding two records of one base cell per thread (the plan's pair lists)
inline bool paired_degrid(const fr_plan *pl) { return !pl->fp64 && pl->vis_per_run >= 4.0; }

// gridder.hip
void plan_build(fr_plan *pl, const double *uvw_m, const double *freq_hz);
int64_t plan_n_keys(const fr_plan *pl);
void plan_export_order(const fr_plan *pl, uint64_t *keys, uint32_t *perm, int64_t *bucket_start);
size_t planes_bytes(const fr_plan *pl);
// arena scratch (bytes, regions rounded) that one call takes at most
size_t degrid_scratch(const fr_plan *pl);
size_t grid_scratch(const fr_plan *pl);
size_t psf_grid_scratch_bound(const fr_plan *pl);
size_t psf_build_scratch(const fr_plan *pl);
size_t psf_plan_device_bound(const fr_plan *pl);
size_t rnr_approx_scratch(const fr_psf *psf, int64_t B);
size_t periodic_conv_scratch(int64_t n_img, int64_t nx, int64_t ny, bool fp64);
size_t rnr_exact_scratch(const fr_plan *pl);
size_t lik_scratch(const fr_plan *pl, const fr_psf *psf, int mode, int64_t B, bool prior);
size_t cg_scratch(const fr_plan *pl, const fr_psf *psf, bool prior);
// vis = R img, or diag(weight) R img when weight is given.  sorted_out: write, in
// the plan's record order, weight times the interpolated plane values without the
// centring phase and conjugation (what grid with sorted_in takes back: the two
// cancel between R and R^+), for R^+ N^-1 R without visibilities in input order.
template <typename T>
void degrid(const fr_plan *pl, const T *img, c2<T> *vis, hipStream_t st, const T *weight = nullptr,
            bool sorted_out = false);
template <typename T>
void grid(const fr_plan *pl, const c2<T> *vis, const T *weight, T *img, hipStream_t st, bool sorted_in = false);

// psf.hip
template <typename T>
void make_psf(fr_plan *pl, const T *weight, double eps_noise, fr_psf *out, hipStream_t st);

// lik.hip
template <typename T>
void apply_rnr_exact(const fr_plan *pl, const T *weight, const T *x, T *y, int64_t B, hipStream_t st);
template <typename T>
void likelihood_grad(const fr_plan *pl, const fr_psf *psf, int mode, const T *s, const T *i_fixed, const void *data,
                     const T *weight, const T *inv_power, int64_t B, T *grad, double *H, hipStream_t st);

// cg.hip
template <typename T>
void cg_solve(const fr_plan *pl, const fr_psf *psf, const T *weight, const T *inv_power, const T *diag, const T *b,
              T *x, int maxiter, double rtol, double *hist, int *iters_done, hipStream_t st);

template <typename T>
void mgvi_metric_apply(const fr_psf *psf, const T *power, const T *diag, const T *x, T *y, hipStream_t st);
template <typename T>
void mgvi_draw(const fr_psf *psf, const T *power, const T *diag, const T *eta0, const T *eta1, T *xi,
               hipStream_t st);
template <typename T>
void mgvi_solve(const fr_psf *psf, const T *power, const T *diag, const T *b, T *x, int maxiter, double rtol,
                double *hist, int *iters_done, hipStream_t st);

// cf.hip
void cf_build(fr_cf *cf);
size_t cf_scratch(const fr_cf *cf);
template <typename T>
void cf_power(const fr_cf *cf, const double *prior, const double *xi_h, const double *xi_v, const double *xi_y,
              T *power, hipStream_t st);
template <typename T>
void cf_logsky(const fr_cf *cf, const T *power, double offset, const T *xi, T *s, int64_t n_img, hipStream_t st);

// psfconv.hip
template <typename T>
void apply_rnr_approx(const fr_psf *psf, const T *x, T *y, int64_t B, hipStream_t st);
// ws: caller-provided workspace of rnr_approx_scratch(psf, B) bytes, or NULL for the
// stream's arena
template <typename T>
void apply_rnr_approx_ex(const fr_psf *psf, const T *x, const T *d_in, T *y, const T *d_out, const T *add,
                         int64_t B, hipStream_t st, void *ws = nullptr);
template <typename T>
void periodic_conv(const Ctx &ctx, const T *x, T *y, int64_t n_img, int64_t nx, int64_t ny, const T *K, int nk,
                   int mode, hipStream_t st);
template <typename T>
void periodic_conv_ex(const Ctx &ctx, const T *x, const T *d_in, T *y, const T *d_out, const T *add,
                      int64_t n_img, int64_t nx, int64_t ny, const T *K, int nk, int mode, hipStream_t st);
template <typename T>
void fft2_inplace(const Ctx &ctx, c2<T> *data, int64_t batch, int64_t n0, int64_t n1, int sign, hipStream_t st);
template <typename T>
void reduce_psf(const fr_psf *in, int64_t hx, int64_t hy, fr_psf *out, hipStream_t st);
int64_t reduced_pad(int64_t n);

}  // namespace frmi
