// Elementwise and reduction kernels shared by the likelihood, CG and PSF code.
// Reductions accumulate in FP64 and are deterministic: each block writes one
// partial sum, and a single block adds the partials in a fixed order.
#pragma once

#include "common.h"

namespace frmi {

constexpr int kRedThreads = 256;
constexpr int kRedMaxBlocks = 1024;  // partial sums per image of a reduction, at most

// Blocks for a reduction over n elements: enough that every thread has about
// four elements (all CUs busy, four loads in flight per thread), at most
// kRedMaxBlocks.
inline int red_blocks(int64_t n) {
    const int64_t b = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), kRedMaxBlocks);
}

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

// This thread's share of sum_i f(i) over a grid-stride loop, four indices per
// step so that their loads are in flight together.  f may also store (each
// index is visited once).  The order of the additions depends only on n and
// the launch shape, so results are reproducible.
template <class F> __device__ __forceinline__ double grid_stride_sum(int64_t n, F f) {
    const int64_t stride = (int64_t)gridDim.x * kRedThreads;
    int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    double s = 0;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const double a0 = f(i), a1 = f(i + stride), a2 = f(i + 2 * stride), a3 = f(i + 3 * stride);
        s += (a0 + a1) + (a2 + a3);
    }
    for (; i < n; i += stride) s += f(i);
    return s;
}

// Sum of n partials by the whole block (thread t adds partials t, t + 256, ...,
// then a block tree); valid in thread 0.  Coherent loads: the partials may have
// been written by other blocks of the same launch.
__device__ __forceinline__ double block_sum_partials(const double *partials, int n) {
    double s = 0;
    for (int k = threadIdx.x; k < n; k += kRedThreads)
        s += __hip_atomic_load(partials + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(s);
}

// partials[img * gridDim.x + blockIdx.x] = this block's share of sum a * b over
// image img (b == nullptr: a * a)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot_partials(const T *__restrict__ a, const T *__restrict__ b,
                                                              int64_t n_per_img, double *__restrict__ partials) {
    const int64_t img = blockIdx.y;
    const T *pa = a + img * n_per_img;
    const T *pb = b ? b + img * n_per_img : pa;
    double s = grid_stride_sum(n_per_img, [&](int64_t i) { return (double)pa[i] * (double)pb[i]; });
    s = block_sum(s);
    if (threadIdx.x == 0) partials[img * gridDim.x + blockIdx.x] = s;
}

// out[img] = (accumulate ? out[img] : 0) + scale * sum of the image's partials;
// one block per image
static __global__ __launch_bounds__(kRedThreads) void k_finish_sums(const double *__restrict__ partials, int nparts,
                                                                    double scale, int accumulate,
                                                                    double *__restrict__ out) {
    const int64_t img = blockIdx.x;
    const double s = block_sum_partials(partials + img * nparts, nparts);
    if (threadIdx.x == 0) out[img] = (accumulate ? out[img] : 0.0) + scale * s;
}

// out[img] = scale * sum_i a_img[i] b_img[i], FP64 accumulation; images of n_per_img elements
template <typename T>
void batched_dot(const T *a, const T *b, int64_t n_per_img, int64_t n_img, double scale, int accumulate,
                 double *out, double *partials /* n_img * kRedMaxBlocks */, hipStream_t st) {
    if (n_img <= 0) return;
    const int nb = red_blocks(n_per_img);
    k_dot_partials<T><<<dim3((unsigned)nb, (unsigned)n_img), kRedThreads, 0, st>>>(a, b, n_per_img, partials);
    LAUNCH_CHECK();
    k_finish_sums<<<dim3((unsigned)n_img), kRedThreads, 0, st>>>(partials, nb, scale, accumulate, out);
    LAUNCH_CHECK();
}

// q mod n for 0 <= q < 2^52 without a 64-bit integer division (inv_n = 1 / n):
// the quotient from the FP64 product is off by at most one, which the two
// comparisons correct
__device__ __forceinline__ int64_t mod_nonneg(int64_t q, int64_t n, double inv_n) {
    const int64_t k = (int64_t)((double)q * inv_n);
    int64_t r = q - k * n;
    if (r < 0) r += n;
    else if (r >= n) r -= n;
    return r;
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
