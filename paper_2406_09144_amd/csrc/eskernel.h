// Exponential-of-semicircle (ES) gridding kernel: host-side parameter choice and
// Fourier-transform corrections, in FP64.
//
// The kernel (Barnett, Magland & af Klinteberg 2019) over a support of W cells is
//   psi(t) = phi(2 t / W),  phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1, else 0,
// and gridding with it is undone in image space by dividing by its Fourier
// transform
//   Psi(xi) = int psi(t) exp(2 pi i t xi) dt
//           = (W/2) int_{-pi/2}^{pi/2} exp(beta (cos th - 1)) cos(pi W xi sin th) cos th d th
// (substituting z = sin th removes the square-root edge singularity so that
// Gauss-Legendre quadrature converges quickly).  With oversampling sigma the image
// samples xi in [-1/(2 sigma), 1/(2 sigma)]; aliasing adds the images Psi(xi + m),
// m != 0, so  E = max_xi sum_{m != 0} |Psi(xi + m)| / Psi(xi)  bounds the relative
// error one dimension contributes.
#pragma once

#include <cmath>
#include <vector>

namespace frmi {

struct ESKernel {
    int W = 0;
    double beta = 0;
    std::vector<double> th, wt;  // quadrature nodes/weights in theta

    ESKernel() = default;
    ESKernel(int W_, double beta_, int nq = 0) : W(W_), beta(beta_) {
        if (nq == 0) nq = 64 + 24 * W;
        gauss_legendre(nq);
    }

    void gauss_legendre(int n) {
        th.resize(n);
        wt.resize(n);
        const double pi = 3.14159265358979323846;
        for (int i = 0; i < n; ++i) {
            double x = std::cos(pi * (i + 0.75) / (n + 0.5));
            double dp = 0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1, p1 = x;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (x * p1 - p0) / (x * x - 1);
                double dx = p1 / dp;
                x -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
            // recompute derivative at the converged node
            double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1);
            th[i] = 0.5 * pi * x;
            wt[i] = 0.5 * pi * 2.0 / ((1 - x * x) * dp * dp);
        }
    }

    double phi(double z) const {
        if (std::fabs(z) > 1) return 0;
        return std::exp(beta * (std::sqrt(1 - z * z) - 1));
    }

    double psi_hat(double xi) const {
        const double pi = 3.14159265358979323846;
        double s = 0;
        for (size_t k = 0; k < th.size(); ++k)
            s += wt[k] * std::exp(beta * (std::cos(th[k]) - 1)) * std::cos(pi * W * xi * std::sin(th[k])) *
                 std::cos(th[k]);
        return 0.5 * W * s;
    }

    // aliasing bound for image coordinates |xi| <= xmax
    double alias_bound(double xmax, int mmax = 10, int nxi = 48) const {
        double worst = 0;
        for (int q = 0; q <= nxi; ++q) {
            double xi = xmax * q / nxi;
            double main = psi_hat(xi);
            double al = 0;
            for (int m = 1; m <= mmax; ++m) al += std::fabs(psi_hat(xi + m)) + std::fabs(psi_hat(xi - m));
            worst = std::max(worst, al / main);
        }
        return worst;
    }
};

// Shape parameter for 2x oversampling: beta = 2.30 W (Barnett et al. 2019).
inline double es_beta(int W) { return 2.30 * W; }

// alias_bound(0.25) of the kernel with beta = 2.30 W, for W = 3 .. 16, evaluated
// once with 3000 quadrature nodes and |m| <= 10 (the evaluation is too slow to
// repeat at every plan creation).
constexpr double kESAliasBound[17] = {
    1.0, 1.0, 1.0, 2.845e-02, 3.723e-03, 3.990e-04, 3.346e-05, 2.879e-06, 4.178e-07,
    5.567e-08, 7.736e-09, 9.073e-10, 8.355e-11, 8.007e-12, 1.010e-12, 1.533e-13, 6.200e-14};

// The kernel along w may use a finer grid than 2x oversampling: with plane spacing
// dw and |t| <= h over the image, the w-image coordinate xi = t dw stays within
// xmax = h dw.  For each support Ww = 4 .. 16 and xmax in kESwXmax: the shape
// beta / Ww minimising alias_bound(xmax) and that bound (gen_es_wtable.py, 1000 +
// 100 Ww quadrature nodes).  A smaller xmax (more planes per unit of w) lets a
// narrower kernel meet the same bound, which pays when the w-range spans few
// planes.
constexpr double kESwXmax[5] = {0.25, 0.2, 0.15, 0.1, 0.05};
struct ESwEntry {
    double beta_over_w, bound;
};
constexpr ESwEntry kESwTable[17][5] = {
    {}, {}, {}, {},
    {{2.20, 1.515e-03}, {2.35, 7.574e-04}, {2.55, 4.021e-04}, {2.70, 2.299e-04}, {2.75, 1.702e-04}},  // Ww = 4
    {{2.25, 1.899e-04}, {2.40, 7.772e-05}, {2.55, 3.861e-05}, {2.75, 1.453e-05}, {2.90, 7.807e-06}},  // Ww = 5
    {{2.25, 2.895e-05}, {2.45, 7.385e-06}, {2.60, 2.957e-06}, {2.75, 1.180e-06}, {2.90, 5.680e-07}},  // Ww = 6
    {{2.30, 2.879e-06}, {2.45, 7.751e-07}, {2.60, 2.717e-07}, {2.75, 9.360e-08}, {2.95, 2.720e-08}},  // Ww = 7
    {{2.30, 4.178e-07}, {2.45, 8.932e-08}, {2.55, 2.041e-08}, {2.70, 5.047e-09}, {2.95, 1.578e-09}},  // Ww = 8
    {{2.25, 4.807e-08}, {2.40, 7.954e-09}, {2.55, 1.702e-09}, {2.80, 3.388e-10}, {2.90, 7.943e-11}},  // Ww = 9
    {{2.25, 5.826e-09}, {2.40, 9.154e-10}, {2.65, 1.299e-10}, {2.75, 2.054e-11}, {2.90, 5.248e-12}},  // Ww = 10
    {{2.25, 8.563e-10}, {2.45, 7.947e-11}, {2.60, 9.097e-12}, {2.75, 1.448e-12}, {2.90, 2.920e-13}},  // Ww = 11
    {{2.30, 8.355e-11}, {2.45, 6.417e-12}, {2.65, 7.760e-13}, {2.75, 1.138e-13}, {2.90, 2.098e-14}},  // Ww = 12
    {{2.30, 8.012e-12}, {2.45, 6.579e-13}, {2.60, 6.964e-14}, {2.75, 1.150e-14}, {2.95, 6.410e-15}},  // Ww = 13
    {{2.30, 1.008e-12}, {2.50, 7.616e-14}, {2.60, 1.165e-14}, {2.75, 5.748e-15}, {2.85, 5.051e-15}},  // Ww = 14
    {{2.30, 1.440e-13}, {2.50, 1.775e-14}, {2.65, 7.867e-15}, {2.60, 5.495e-15}, {3.00, 4.807e-15}},  // Ww = 15
    {{2.30, 4.816e-14}, {2.50, 1.409e-14}, {2.65, 7.894e-15}, {2.60, 5.497e-15}, {2.55, 4.666e-15}},  // Ww = 16
};

// Smallest support whose per-dimension bound, summed over `dims` dimensions,
// stays below epsilon (W >= wmin).
inline int es_support(double epsilon, int dims, int wmin = 4) {
    for (int W = wmin; W <= 16; ++W)
        if (dims * kESAliasBound[W] <= epsilon) return W;
    return 16;
}

}  // namespace frmi
