// Elementwise and reduction kernels shared by the likelihood, CG and PSF code.
// Reductions accumulate in FP64 and are deterministic: each block writes one
// partial sum, and a single block adds the partials in a fixed order.
#pragma once

#include "common.h"

namespace frmi {

constexpr int kRedThreads = 256;
constexpr int kRedBlocksPerImage = 64;  // partials per image of a batched reduction

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[kRedThreads / 64];
    // wavefront reduction (64 lanes)
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kRedThreads / 64; ++k) t += sh[k];
    return t;  // valid in thread 0
}

// partials[img * kRedBlocksPerImage + blockIdx.x] = sum over image img of a * b (b == nullptr: a * a)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot_partials(const T *__restrict__ a, const T *__restrict__ b,
                                                              int64_t n_per_img, double *__restrict__ partials) {
    const int64_t img = blockIdx.y;
    const T *pa = a + img * n_per_img;
    const T *pb = b ? b + img * n_per_img : pa;
    double s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n_per_img;
         i += (int64_t)gridDim.x * kRedThreads)
        s += (double)pa[i] * (double)pb[i];
    s = block_sum(s);
    if (threadIdx.x == 0) partials[img * gridDim.x + blockIdx.x] = s;
}

// out[img] = (accumulate ? out[img] : 0) + scale * sum of the image's partials
static __global__ void k_finish_sums(const double *__restrict__ partials, int nparts, int64_t n_img, double scale,
                              int accumulate, double *__restrict__ out) {
    const int64_t img = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (img >= n_img) return;
    double s = 0;
    for (int k = 0; k < nparts; ++k) s += partials[img * nparts + k];
    out[img] = (accumulate ? out[img] : 0.0) + scale * s;
}

// out[img] = scale * sum_i a_img[i] b_img[i], FP64 accumulation; images of n_per_img elements
template <typename T>
void batched_dot(const T *a, const T *b, int64_t n_per_img, int64_t n_img, double scale, int accumulate,
                 double *out, double *partials /* n_img * kRedBlocksPerImage */, hipStream_t st) {
    if (n_img <= 0) return;
    k_dot_partials<T><<<dim3(kRedBlocksPerImage, (unsigned)n_img), kRedThreads, 0, st>>>(a, b, n_per_img, partials);
    LAUNCH_CHECK();
    k_finish_sums<<<dim3((unsigned)((n_img + 63) / 64)), 64, 0, st>>>(partials, kRedBlocksPerImage, n_img, scale,
                                                                      accumulate, out);
    LAUNCH_CHECK();
}

// generic grid-stride elementwise launcher
template <class F> __global__ void k_map(F f, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        f(i);
}

template <class F> void map_async(F f, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    k_map<F><<<dim3((unsigned)blocks), 256, 0, st>>>(f, n);
    LAUNCH_CHECK();
}

}  // namespace frmi
