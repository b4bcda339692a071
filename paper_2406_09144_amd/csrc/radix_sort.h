// Stable least-significant-digit radix sort of (64-bit key, 32-bit value) pairs,
// used by the plan to order visibilities by (channel, first w-plane, uv tile,
// base cell inside the tile).
//
// One pass per 8-bit digit of the key bits [0, end_bit):
//   1. k_radix_hist:    each workgroup counts the digits of its tile of
//                       kRadixTile consecutive keys into LDS and writes the 256
//                       counts to a digit-major table, hist[digit][tile];
//   2. exclusive scan of that table (k_scan_chunks, k_scan_totals,
//                       k_scan_apply), so that entry (digit, tile) becomes the
//                       first output position of the tile's keys with that digit:
//                       all smaller digits come first, and within a digit the
//                       earlier tiles;
//   3. k_radix_scatter: each workgroup walks its tile again in input order, in
//                       rounds of one key per thread, and gives every key its
//                       rank among the equal digits before it: inside a
//                       wavefront from eight ballots (one per digit bit: the
//                       lanes whose digits agree on every bit), across the
//                       wavefronts of a round and across rounds from LDS
//                       counters.  Equal digits keep their input order, which
//                       makes each pass, and hence the sort, stable.
// The passes alternate between the two buffer pairs; the result is in the pair
// the last pass wrote.  Every step is deterministic (no global atomics).
#pragma once

#include "common.h"

namespace frmi {

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;                               // keys per thread and tile
constexpr int kRadixTile = kRadixThreads * kRadixItems;      // keys per workgroup
constexpr int kScanThreads = 256;
constexpr int kScanChunk = 4096;                              // table entries per scan workgroup

__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                              int shift, int n_tiles,
                                                              uint32_t *__restrict__ hist) {
    __shared__ uint32_t cnt[kRadixBins];
    cnt[threadIdx.x] = 0;  // kRadixThreads == kRadixBins
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int r = 0; r < kRadixItems; ++r) {
        const int64_t i = base + r * kRadixThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & (kRadixBins - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = cnt[threadIdx.x];
}

// sum of each chunk of kScanChunk entries
__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(const uint32_t *__restrict__ a, int64_t n,
                                                              uint64_t *__restrict__ chunk_sum) {
    __shared__ uint64_t sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    uint64_t s = 0;
    for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads)
        if (base + k < n) s += a[base + k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t += sh[w];
        chunk_sum[blockIdx.x] = t;
    }
}

// exclusive scan of the chunk sums, in place (one workgroup, sequential per thread
// over a contiguous share, then a scan of the shares)
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(uint64_t *__restrict__ chunk_sum, int64_t n_chunks) {
    __shared__ uint64_t part[kScanThreads];
    const int64_t per = (n_chunks + kScanThreads - 1) / kScanThreads;
    const int64_t b = threadIdx.x * per, e = min(n_chunks, b + per);
    uint64_t s = 0;
    for (int64_t k = b; k < e; ++k) s += chunk_sum[k];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int t = 0; t < kScanThreads; ++t) {
            const uint64_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    uint64_t run = part[threadIdx.x];
    for (int64_t k = b; k < e; ++k) {
        const uint64_t v = chunk_sum[k];
        chunk_sum[k] = run;
        run += v;
    }
}

// exclusive scan inside each chunk plus the chunk's offset: a[i] -> position (in place, as 64-bit)
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t *__restrict__ a, int64_t n,
                                                             const uint64_t *__restrict__ chunk_off,
                                                             uint64_t *__restrict__ out) {
    constexpr int PER = kScanChunk / kScanThreads;  // 16 contiguous entries per thread
    __shared__ uint64_t part[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * PER;
    uint32_t v[PER];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = base + k < n ? a[base + k] : 0u;
        s += v[k];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread sums
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint64_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = chunk_off[blockIdx.x] + part[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// lanes of this wavefront whose digit equals this lane's digit
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t ones = __ballot(valid && ((d >> b) & 1u));
        m &= ((d >> b) & 1u) ? ones : ~ones;
    }
    return m;
}

__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const uint64_t *__restrict__ keys_in,
                                                                 const uint32_t *__restrict__ vals_in, int64_t n,
                                                                 int shift, int n_tiles,
                                                                 const uint64_t *__restrict__ pos,
                                                                 uint64_t *__restrict__ keys_out,
                                                                 uint32_t *__restrict__ vals_out) {
    constexpr int NW = kRadixThreads / 64;
    __shared__ uint64_t start[kRadixBins];       // next output position per digit
    __shared__ uint32_t wcnt[NW][kRadixBins];    // keys per (wavefront, digit) this round
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    start[threadIdx.x] = pos[(int64_t)threadIdx.x * n_tiles + blockIdx.x];
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixItems; ++r) {
        const int64_t i = base + r * kRadixThreads + threadIdx.x;
        const bool valid = i < n;
        uint64_t k = 0;
        uint32_t v = 0, d = 0;
        if (valid) {
            k = keys_in[i];
            v = vals_in[i];
            d = (uint32_t)(k >> shift) & (kRadixBins - 1);
        }
        const uint64_t m = match_digit(d, valid);
        const uint32_t rank = (uint32_t)__popcll(m & below);
        // the lowest lane of each digit group records the group's size
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint64_t p = start[d] + rank;
            for (int w = 0; w < wave; ++w) p += wcnt[w][d];
            keys_out[p] = k;
            vals_out[p] = v;
        }
        __syncthreads();
        // advance the per-digit positions by this round's keys and clear the counts
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            tot += wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = 0;
        }
        start[threadIdx.x] += tot;
        __syncthreads();
    }
}

// Device buffers of one sort: the ping-pong pairs and the scan tables.
struct RadixSortBuffers {
    size_t bytes(int64_t n) const {
        const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
        const int64_t entries = tiles * kRadixBins;
        const int64_t chunks = (entries + kScanChunk - 1) / kScanChunk;
        return (size_t)entries * (4 + 8) + (size_t)chunks * 8;
    }
};

// Sort (k0, v0) by key bits [0, end_bit), stably.  k1/v1 are buffers of the same
// size; tmp holds RadixSortBuffers().bytes(n).  Returns true when the result is in
// (k1, v1), false when in (k0, v0).
inline bool radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int end_bit,
                             void *tmp, hipStream_t st) {
    if (n <= 1 || end_bit <= 0) return false;
    const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
    FR_REQUIRE(tiles < (int64_t(1) << 31), "too many keys to sort");
    const int64_t entries = tiles * kRadixBins;
    const int64_t chunks = (entries + kScanChunk - 1) / kScanChunk;
    uint32_t *hist = (uint32_t *)tmp;
    uint64_t *pos = (uint64_t *)(hist + entries);
    uint64_t *csum = pos + entries;
    bool flipped = false;
    for (int shift = 0; shift < end_bit; shift += kRadixBits) {
        uint64_t *ki = flipped ? k1 : k0, *ko = flipped ? k0 : k1;
        uint32_t *vi = flipped ? v1 : v0, *vo = flipped ? v0 : v1;
        k_radix_hist<<<dim3((unsigned)tiles), kRadixThreads, 0, st>>>(ki, n, shift, (int)tiles, hist);
        LAUNCH_CHECK();
        k_scan_chunks<<<dim3((unsigned)chunks), kScanThreads, 0, st>>>(hist, entries, csum);
        LAUNCH_CHECK();
        k_scan_totals<<<1, kScanThreads, 0, st>>>(csum, chunks);
        LAUNCH_CHECK();
        k_scan_apply<<<dim3((unsigned)chunks), kScanThreads, 0, st>>>(hist, entries, csum, pos);
        LAUNCH_CHECK();
        k_radix_scatter<<<dim3((unsigned)tiles), kRadixThreads, 0, st>>>(ki, vi, n, shift, (int)tiles, pos, ko, vo);
        LAUNCH_CHECK();
        flipped = !flipped;
    }
    return flipped;
}

}  // namespace frmi
