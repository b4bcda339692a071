/*
 * FP64 oracle: direct (brute-force) sums for the interferometric response.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that the HIP
 * path is checked against.  It shares no code with the HIP library and nothing in
 * the product path may link or call it.
 *
 * Conventions (fast-resolve, Sec. 2, eq. "rime", with scalar gains G = 1, the
 * integral written as a sum over pixels, image in flux per pixel):
 *   l_i = (i - nx/2) dx,  m_j = (j - ny/2) dy,  n_ij = sqrt(1 - l_i^2 - m_j^2)
 *   R:   V_k  = sum_ij I_ij a_ij exp(-2 pi i [u_k l_i + v_k m_j + w_k (n_ij - 1)])
 *   R^+: X_ij = a_ij Re sum_k y_k exp(+2 pi i [u_k l_i + v_k m_j + w_k (n_ij - 1)])
 * with a_ij = 1/n_ij when divide_by_n is set (the 1/sqrt(1 - l^2) factor of the
 * w-term C(l, w) in Sec. 2), else 1.  u, v, w are in wavelengths.  The phase is
 * formed in cycles, reduced to [-1/2, 1/2], and only then multiplied by 2 pi.
 *
 * Parity pins for this file live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>

static const double TWO_PI = 6.283185307179586476925286766559;

/* n - 1 written as -(l^2 + m^2) / (1 + n): the same number as sqrt(...) - 1,
 * without the cancellation of subtracting 1 from a value close to 1. */
static double n_minus_1(double l, double m)
{
    double r2 = l * l + m * m;
    return -r2 / (1.0 + sqrt(1.0 - r2));
}

static double reduce_cycles(double c)
{
    return c - nearbyint(c);
}

/* R (degridding by definition): img [nx][ny] -> vis [nvis][2] (re, im). */
void oracle_degrid(int64_t nx, int64_t ny, double dx, double dy, int divide_by_n,
                   const double *img, int64_t nvis,
                   const double *u, const double *v, const double *w, double *vis)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < nvis; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t i = 0; i < nx; ++i) {
            double l = (double)(i - nx / 2) * dx;
            for (int64_t j = 0; j < ny; ++j) {
                double x = img[i * ny + j];
                if (x == 0.0) continue;
                double m = (double)(j - ny / 2) * dy;
                double nm1 = n_minus_1(l, m);
                double amp = divide_by_n ? x / (1.0 + nm1) : x;
                double ph = reduce_cycles(u[k] * l + v[k] * m + w[k] * nm1);
                re += amp * cos(TWO_PI * ph);
                im -= amp * sin(TWO_PI * ph);
            }
        }
        vis[2 * k] = re;
        vis[2 * k + 1] = im;
    }
}

/* R^+ at a list of flat pixel indices (i * ny + j); vis may carry weights already. */
void oracle_grid_pixels(int64_t nx, int64_t ny, double dx, double dy, int divide_by_n,
                        int64_t nvis, const double *u, const double *v, const double *w,
                        const double *vis, int64_t npix, const int64_t *pix, double *out)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npix; ++p) {
        int64_t i = pix[p] / ny, j = pix[p] % ny;
        double l = (double)(i - nx / 2) * dx;
        double m = (double)(j - ny / 2) * dy;
        double nm1 = n_minus_1(l, m);
        double acc = 0.0;
        for (int64_t k = 0; k < nvis; ++k) {
            double ph = reduce_cycles(u[k] * l + v[k] * m + w[k] * nm1);
            /* Re[(a + ib)(cos + i sin)] = a cos - b sin */
            acc += vis[2 * k] * cos(TWO_PI * ph) - vis[2 * k + 1] * sin(TWO_PI * ph);
        }
        out[p] = divide_by_n ? acc / (1.0 + nm1) : acc;
    }
}

/* R^+ on every pixel. */
void oracle_grid(int64_t nx, int64_t ny, double dx, double dy, int divide_by_n,
                 int64_t nvis, const double *u, const double *v, const double *w,
                 const double *vis, double *img)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nx; ++i) {
        double l = (double)(i - nx / 2) * dx;
        for (int64_t j = 0; j < ny; ++j) {
            double m = (double)(j - ny / 2) * dy;
            double nm1 = n_minus_1(l, m);
            double acc = 0.0;
            for (int64_t k = 0; k < nvis; ++k) {
                double ph = reduce_cycles(u[k] * l + v[k] * m + w[k] * nm1);
                acc += vis[2 * k] * cos(TWO_PI * ph) - vis[2 * k + 1] * sin(TWO_PI * ph);
            }
            img[i * ny + j] = divide_by_n ? acc / (1.0 + nm1) : acc;
        }
    }
}

/* Coplanar PSF on the doubled grid (Sec. 3.3.2: the PSF must cover twice the
 * field of view):  PSF0[i][j] = sum_k wt_k cos(2 pi [u_k (i-nx) dx + v_k (j-ny) dy])
 * for i in [0, 2nx), j in [0, 2ny); the peak sits at (nx, ny). */
void oracle_psf0(int64_t nx, int64_t ny, double dx, double dy, int64_t nvis,
                 const double *u, const double *v, const double *wt, double *psf)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < 2 * nx; ++i) {
        double l = (double)(i - nx) * dx;
        for (int64_t j = 0; j < 2 * ny; ++j) {
            double m = (double)(j - ny) * dy;
            double acc = 0.0;
            for (int64_t k = 0; k < nvis; ++k)
                acc += wt[k] * cos(TWO_PI * reduce_cycles(u[k] * l + v[k] * m));
            psf[i * 2 * ny + j] = acc;
        }
    }
}

/* Brute-force linear convolution with the doubled-grid PSF:
 *   y_ij = sum_{i'j'} PSF0[nx + i - i'][ny + j - j'] x_{i'j'},   0 <= i, i' < nx.
 * Optional output pixel subset (pix != 0): y has npix entries. */
void oracle_psf_conv_direct(int64_t nx, int64_t ny, const double *psf0, const double *x,
                            int64_t npix, const int64_t *pix, double *y)
{
    int64_t nout = pix ? npix : nx * ny;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < nout; ++p) {
        int64_t o = pix ? pix[p] : p;
        int64_t i = o / ny, j = o % ny;
        double acc = 0.0;
        for (int64_t ii = 0; ii < nx; ++ii) {
            const double *prow = psf0 + (nx + i - ii) * 2 * ny + (ny + j);
            const double *xrow = x + ii * ny;
            for (int64_t jj = 0; jj < ny; ++jj)
                acc += prow[-jj] * xrow[jj];
        }
        y[p] = acc;
    }
}
