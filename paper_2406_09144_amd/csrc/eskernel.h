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

// Smallest support whose per-dimension bound, summed over `dims` dimensions,
// stays below epsilon (W >= wmin).
inline int es_support(double epsilon, int dims, int wmin = 4) {
    for (int W = wmin; W <= 16; ++W)
        if (dims * kESAliasBound[W] <= epsilon) return W;
    return 16;
}

}  // namespace frmi
