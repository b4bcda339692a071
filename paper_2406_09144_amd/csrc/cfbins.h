// Frequency bins of the correlated-field amplitude model (host-only C++, no HIP):
// the distinct non-zero |k|^2 of an nx x ny grid in integer frequency units (the
// order of numpy's fftfreq times n), their multiplicity over the full grid, the
// log-frequencies t = ln|k| with their steps d (d_0 = 0), and the bin of every
// cell of the r2c half spectrum [nx][ny/2 + 1] (-1 at k = 0).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <vector>

namespace frmi {

struct CFBins {
    std::vector<int64_t> k2;     // [J] ascending
    std::vector<double> mult;    // [J]
    std::vector<double> t, d;    // [J]
    std::vector<int32_t> bin;    // [nx][ny/2 + 1]
};

inline CFBins cf_bins_host(int64_t nx, int64_t ny) {
    if (nx < 2 || ny < 2) throw std::invalid_argument("grid too small for the amplitude model");
    const int64_t h = ny / 2 + 1;
    auto fk = [](int64_t i, int64_t n) { return i < (n + 1) / 2 ? i : i - n; };
    std::vector<int64_t> k2full((size_t)(nx * ny));
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < ny; ++j) {
            const int64_t a = fk(i, nx), b = fk(j, ny);
            k2full[(size_t)(i * ny + j)] = a * a + b * b;
        }
    CFBins out;
    out.k2 = k2full;
    std::sort(out.k2.begin(), out.k2.end());
    out.k2.erase(std::unique(out.k2.begin(), out.k2.end()), out.k2.end());
    out.k2.erase(out.k2.begin());  // k = 0 is the zero mode
    const int64_t J = (int64_t)out.k2.size();
    auto bin_of = [&](int64_t k2) -> int32_t {
        if (k2 == 0) return -1;
        return (int32_t)(std::lower_bound(out.k2.begin(), out.k2.end(), k2) - out.k2.begin());
    };
    out.mult.assign((size_t)J, 0.0);
    for (int64_t k2 : k2full)
        if (k2) out.mult[(size_t)bin_of(k2)] += 1.0;
    out.t.resize((size_t)J);
    out.d.resize((size_t)J);
    for (int64_t j = 0; j < J; ++j) {
        out.t[(size_t)j] = 0.5 * std::log((double)out.k2[(size_t)j]);
        out.d[(size_t)j] = j ? out.t[(size_t)j] - out.t[(size_t)(j - 1)] : 0.0;
    }
    out.bin.resize((size_t)(nx * h));
    for (int64_t i = 0; i < nx; ++i)
        for (int64_t j = 0; j < h; ++j) out.bin[(size_t)(i * h + j)] = bin_of(k2full[(size_t)(i * ny + j)]);
    return out;
}

}  // namespace frmi
