// Host-only logic of the library checked under AddressSanitizer and
// UndefinedBehaviorSanitizer (built with g++, no GPU):
//   * the ES-kernel quadrature: Gauss-Legendre nodes integrate polynomials
//     exactly; the Fourier transform psi_hat(0) equals the integral of the kernel
//     by a fine midpoint rule; psi_hat is even; the aliasing bound of W = 5..8
//     with beta = 2.30 W matches the table the plans use (computed once with 3000
//     nodes) to 5%; the support chosen for an epsilon meets it; the w-kernel
//     table (finer w-grids) spot-checked the same way, its shapes local minima;
//   * the amplitude-model bins: every non-zero frequency of the full grid counted
//     once, the half-spectrum map pointing at the bin of its |k|^2, ascending
//     log-frequencies with steps that sum to the span.
// Prints "host checks ok" and exits 0, or names the failed check and exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "../../paper_2406_09144_amd/csrc/cfbins.h"
#include "../../paper_2406_09144_amd/csrc/eskernel.h"

static int failures = 0;
#define CHECK(cond, ...)                               \
    do {                                               \
        if (!(cond)) {                                 \
            std::printf("FAILED: " __VA_ARGS__);       \
            std::printf("\n");                         \
            ++failures;                                \
        }                                              \
    } while (0)

static void check_eskernel() {
    const double pi = 3.14159265358979323846;
    // nodes th in [-pi/2, pi/2]: sum wt th^k = integral of th^k
    frmi::ESKernel k(7, frmi::es_beta(7), 40);
    for (int p = 0; p <= 10; ++p) {
        double s = 0;
        for (size_t i = 0; i < k.th.size(); ++i) s += k.wt[i] * std::pow(k.th[i], p);
        const double exact = (p % 2) ? 0.0 : 2.0 * std::pow(pi / 2, p + 1) / (p + 1);
        CHECK(std::fabs(s - exact) <= 1e-12 * (1 + std::fabs(exact)), "Gauss-Legendre moment %d: %g vs %g", p, s,
              exact);
    }
    for (int W : {4, 7, 12}) {
        frmi::ESKernel e(W, frmi::es_beta(W));
        // psi_hat(0) = integral over t in [-W/2, W/2] of phi(2 t / W)
        const int n = 200000;
        double s = 0;
        for (int i = 0; i < n; ++i) {
            const double t = -0.5 * W + (i + 0.5) * W / (double)n;
            s += e.phi(2.0 * t / W) * W / (double)n;
        }
        CHECK(std::fabs(e.psi_hat(0.0) - s) <= 1e-8 * s, "psi_hat(0) W=%d: %.15g vs %.15g", W, e.psi_hat(0.0), s);
        CHECK(std::fabs(e.psi_hat(0.3) - e.psi_hat(-0.3)) <= 1e-14 * e.psi_hat(0.0), "psi_hat even, W=%d", W);
    }
    for (int W = 5; W <= 8; ++W) {
        frmi::ESKernel e(W, frmi::es_beta(W), 3000);
        const double b = e.alias_bound(0.25);
        CHECK(std::fabs(b / frmi::kESAliasBound[W] - 1.0) < 0.05, "alias bound W=%d: %g vs table %g", W, b,
              frmi::kESAliasBound[W]);
    }
    // the w-kernel table: spot checks with 3000 nodes (the shape and the bound)
    const int wws[3] = {5, 6, 8};
    const int xis[3] = {4, 2, 1};
    for (int q = 0; q < 3; ++q) {
        const int Ww = wws[q], xi = xis[q];
        const frmi::ESwEntry e = frmi::kESwTable[Ww][xi];
        frmi::ESKernel k(Ww, e.beta_over_w * Ww, 3000);
        const double b = k.alias_bound(frmi::kESwXmax[xi]);
        CHECK(std::fabs(b / e.bound - 1.0) < 0.05, "w table Ww=%d xmax=%g: %g vs %g", Ww, frmi::kESwXmax[xi], b,
              e.bound);
        // the tabulated shape is no worse than its neighbours on the beta grid
        frmi::ESKernel lo(Ww, (e.beta_over_w - 0.1) * Ww, 3000), hi(Ww, (e.beta_over_w + 0.1) * Ww, 3000);
        CHECK(lo.alias_bound(frmi::kESwXmax[xi]) >= 0.99 * b && hi.alias_bound(frmi::kESwXmax[xi]) >= 0.99 * b,
              "w table shape Ww=%d xmax=%g is not a minimum", Ww, frmi::kESwXmax[xi]);
    }
    for (double eps : {1e-3, 1e-5, 1e-8, 1e-11}) {
        const int W = frmi::es_support(eps, 2);
        CHECK(2 * frmi::kESAliasBound[W] <= eps || W == 16, "support for eps %g", eps);
        CHECK(W == 4 || 2 * frmi::kESAliasBound[W - 1] > eps, "support for eps %g is not the smallest", eps);
    }
}

static void check_cf_bins(int64_t nx, int64_t ny) {
    const frmi::CFBins b = frmi::cf_bins_host(nx, ny);
    const int64_t J = (int64_t)b.k2.size(), h = ny / 2 + 1;
    double total = 0;
    for (double m : b.mult) total += m;
    CHECK(total == (double)(nx * ny - 1), "multiplicities of %lldx%lld sum to %g", (long long)nx, (long long)ny,
          total);
    for (int64_t j = 1; j < J; ++j) CHECK(b.k2[(size_t)j] > b.k2[(size_t)(j - 1)], "bins ascending");
    double dsum = 0;
    for (int64_t j = 0; j < J; ++j) dsum += b.d[(size_t)j];
    CHECK(std::fabs(dsum - (b.t[(size_t)(J - 1)] - b.t[0])) <= 1e-12 * (1 + std::fabs(dsum)), "steps sum to span");
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < h; ++j) {
            const int64_t a = i < (nx + 1) / 2 ? i : i - nx;
            const int64_t k2 = a * a + j * j;
            const int32_t bin = b.bin[(size_t)(i * h + j)];
            if (k2 == 0) {
                CHECK(bin == -1, "zero mode bin");
            } else {
                CHECK(bin >= 0 && bin < J && b.k2[(size_t)bin] == k2, "bin of (%lld, %lld)", (long long)i,
                      (long long)j);
            }
        }
}

int main() {
    check_eskernel();
    check_cf_bins(16, 16);
    check_cf_bins(32, 64);
    check_cf_bins(128, 32);
    if (failures) return 1;
    std::printf("host checks ok\n");
    return 0;
}
