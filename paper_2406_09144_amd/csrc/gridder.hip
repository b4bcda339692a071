// Exact response R (degridding, Sec. 2 Eq. 1) and its adjoint R^+ (gridding,
// Sec. 3.2) at a requested accuracy epsilon: ES-kernel non-uniform FFT on a 2x
// oversampled uv grid, with improved w-stacking (the kernel also runs along w,
// and its Fourier transform in (n - 1) is divided out in image space).
//
// Degridding of channel c:
//   1. rows:    for each w-plane p and image row i, the prepared row
//               img * a / (Psi_u Psi_v Psi_w) * exp(-2 pi i w_p t) is placed into the
//               wrapped grid row and transformed (only the nx non-zero grid rows);
//   2. columns: forward FFT of every grid column (zero rows are not read);
//   3. degrid:  one workgroup per work item (uv tile x first w-plane): the tile and
//               its W-1 halo of each touched plane is staged in LDS, every
//               visibility sums psi_w psi_u psi_v G over its W x W x Ww footprint.
// Gridding is the exact transpose: each wavefront of a work item's workgroup takes
// batches of 64 visibilities (one coalesced load per batch, values broadcast
// lane-to-lane) and spreads each into LDS tiles of the touched planes (lane (a, b)
// owns footprint cell (a, b), so each LDS atomic instruction hits distinct cells);
// every work item stores its tiles as a partial result, an owner-computes pass
// sums the partials covering each plane tile in a fixed order (no global
// atomics, no clearing, deterministic), inverse column FFT (keeping only the
// non-zero rows), then a row kernel that transforms each plane row and
// accumulates Re(exp(+2 pi i w_p t) G) over planes into the image row.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "eskernel.h"
#include "fftk.h"
#include "objects.h"
#include "profiler.h"
#include "radix_sort.h"

namespace frmi {

constexpr double kCLight = 299792458.0;
constexpr int kTile = 32;

// ------------------------------------------------------------------ plan kernels
template <typename T>
__global__ void k_vis_coords(const double *__restrict__ uvw, const double *__restrict__ freq, int64_t n_vis,
                             int n_chan, int log2nu, int log2nv, double dx, double dy, int W, int Ww, int coplanar,
                             double w0, double dw, double yc, double two_pi_h, int taylor, int ntv, int n_tiles,
                             int n_p0,
                             uint32_t *__restrict__ key, uint32_t *__restrict__ idx, uint32_t *__restrict__ cell,
                             T *__restrict__ du, T *__restrict__ dv, T *__restrict__ dwf, T *__restrict__ ph) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vis) return;
    const int64_t row = v / n_chan;
    const int chan = (int)(v - row * n_chan);
    const double f = freq[chan] / kCLight;
    double u = uvw[3 * row] * f, vv = uvw[3 * row + 1] * f, w = coplanar ? 0.0 : uvw[3 * row + 2] * f;
    uint32_t conj = 0;
    if (w < 0) {  // real sky: V(-u,-v,-w) = conj V(u,v,w); keep w >= 0
        u = -u;
        vv = -vv;
        w = -w;
        conj = 1;
    }
    const int nu = 1 << log2nu, nv = 1 << log2nv;
    // grid coordinates in cells, wrapped into [0, n): exact because image pixels
    // sit on integer multiples of the pixel size
    double ku = u * (double)nu * dx;
    ku -= floor(ku / nu) * nu;
    double kv = vv * (double)nv * dy;
    kv -= floor(kv / nv) * nv;
    int a0 = (int)ceil(ku - 0.5 * W);
    const double fu = ku - a0;
    a0 = (a0 + nu) & (nu - 1);
    int b0 = (int)ceil(kv - 0.5 * W);
    const double fv = kv - b0;
    b0 = (b0 + nv) & (nv - 1);
    const int tu = a0 / kTile, tv = b0 / kTile;
    int p0 = 0;
    double fw = 0, phc = 0;
    if (taylor) {
        fw = two_pi_h * w;  // the Taylor variable x = 2 pi w h; every term is a plane
        phc = w * yc;
        phc -= rint(phc);
    } else if (!coplanar) {
        const double kw = (w - w0) / dw;
        p0 = (int)ceil(kw - 0.5 * Ww);
        fw = kw - p0;
        p0 = min(max(p0, 0), n_p0 - 1);
        phc = w * yc;
        phc -= rint(phc);
    }
    key[v] = (uint32_t)(((int64_t)chan * n_p0 + p0) * n_tiles + (int64_t)tu * ntv + tv);
    idx[v] = (uint32_t)v | (conj << 31);
    cell[v] = (uint32_t)(a0 - tu * kTile) | ((uint32_t)(b0 - tv * kTile) << 16);
    du[v] = (T)fu;
    dv[v] = (T)fv;
    dwf[v] = (T)fw;
    ph[v] = (T)phc;
}

// Sort key of a visibility: its bucket (channel, first plane, tile) above the
// position of its base cell inside the tile, so that a bucket's visibilities
// come out grouped by base cell (runs that the gridder accumulates in
// registers).  The radix sort is stable, which makes the record order, and
// hence every summation order, a function of the input alone.
__global__ void k_sort_keys(const uint32_t *__restrict__ key, const uint32_t *__restrict__ cell, int64_t n,
                            uint64_t *__restrict__ k64, uint32_t *__restrict__ perm) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint32_t c = cell[v];
    k64[v] = ((uint64_t)key[v] << 10) | (uint64_t)((c & 0xffffu) * kTile + (c >> 16));
    perm[v] = (uint32_t)v;
}

// offs[k] = first sorted position whose bucket is >= k, for k = 0 .. n_keys
__global__ void k_bucket_bounds(const uint64_t *__restrict__ k64, int64_t n, int64_t n_keys,
                                int64_t *__restrict__ offs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n_keys) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(k64[mid] >> 10) < k) lo = mid + 1;
        else hi = mid;
    }
    offs[k] = lo;
}

// number of sorted records whose (bucket, base cell) differs from the previous
// record's: the runs the gridding spread accumulates, less one
__global__ void k_count_runs(const uint64_t *__restrict__ k64, int64_t n, unsigned long long *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool step = i > 0 && i < n && k64[i] != k64[i - 1];
    const unsigned long long b = __ballot(step);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

// flag[i] = 1 where sorted record i starts a run (its bucket and base cell differ
// from the previous record's, or i = 0), for records first .. first + n - 1
__global__ void k_run_flags(const uint64_t *__restrict__ k64, int64_t first, int64_t n, uint8_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = first + i;
    flag[i] = (j == 0 || k64[j] != k64[j - 1]) ? 1 : 0;
}

// rows of the tile (halo included) that gridding item i touches: its records are
// sorted by base cell, so the first and last hold the smallest and largest
// base row
__global__ void k_item_rows(WorkItem *__restrict__ items, int64_t n_items, const uint32_t *__restrict__ r_cell,
                            int W) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    WorkItem it = items[i];
    const int r0 = (int)(r_cell[it.start] & 0xffffu);
    const int r1 = (int)(r_cell[it.start + it.count - 1] & 0xffffu) + W - 1;
    items[i].rows = r0 | (r1 << 16);
}

template <typename T>
__global__ void k_gather_records(int64_t n, const uint32_t *__restrict__ perm, const uint32_t *__restrict__ i_idx,
                                 const uint32_t *__restrict__ i_cell, const T *__restrict__ i_du,
                                 const T *__restrict__ i_dv, const T *__restrict__ i_dw, const T *__restrict__ i_ph,
                                 uint32_t *__restrict__ o_idx, uint32_t *__restrict__ o_cell, T *__restrict__ o_du,
                                 T *__restrict__ o_dv, T *__restrict__ o_dw, T *__restrict__ o_ph,
                                 uint32_t *__restrict__ o_pos) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const uint32_t v = perm[pos];
    const uint32_t id = i_idx[v];
    o_idx[pos] = id;
    // record position of visibility v (= id & 0x7fffffff), with its conjugation flag
    o_pos[id & 0x7fffffffu] = (uint32_t)pos | (id & 0x80000000u);
    o_cell[pos] = i_cell[v];
    o_du[pos] = i_du[v];
    o_dv[pos] = i_dv[v];
    o_dw[pos] = i_dw[v];
    o_ph[pos] = i_ph[v];
}

// ------------------------------------------------------------------ kernel weights
template <typename T> __device__ __forceinline__ T es_eval(T z, T beta) {
    const T q = T(1) - z * z;
    return q >= T(0) ? (T)exp(beta * (sqrt(q) - T(1))) : T(0);
}
// FP32: the hardware square root and base-2 exponential.  Rounding the argument
// beta (sqrt(q) - 1) (|.| <= beta ~ 2.3 W) to FP32 already costs about 1e-6
// relative in the result, so the correctly rounded library routines buy nothing.
template <> __device__ __forceinline__ float es_eval<float>(float z, float beta) {
    const float q = 1.0f - z * z;
    constexpr float kLog2e = 1.4426950408889634f;
    return q >= 0.0f ? __builtin_amdgcn_exp2f(beta * kLog2e * (__builtin_amdgcn_sqrtf(q) - 1.0f)) : 0.0f;
}

// Weight of plane p for a visibility with w coordinate x: the ES w-kernel at
// x - p (improved w-stacking, x in planes) or the Taylor coefficient x^p / p!
// (x = 2 pi w h).
template <typename T> __device__ __forceinline__ T plane_weight(T x, int p, int Ww, T wbeta, int taylor) {
    if (taylor) {
        T c = T(1);
        for (int j = 1; j <= p; ++j) c *= x / T(j);
        return c;
    }
    return es_eval<T>((x - T(p)) * (T(2) / T(Ww)), wbeta);
}

// ------------------------------------------------------------------ degrid
// One workgroup per degridding item (records of one uv tile and first w-plane);
// the planes' tile is staged in LDS one plane at a time.  Without PAIR, thread j
// interpolates records j, j + NTHR, ... (VPT of them).  With PAIR (VPT = 2),
// thread t takes entry t of the item's pair list (it.rows entries, at most NTHR):
// two consecutive records of one base cell, or one record alone; the two share
// every tile read of the footprint.
template <typename T, int W, int NTHR, int VPT, bool PAIR = false>
__global__ __launch_bounds__(NTHR) void k_degrid(const WorkItem *__restrict__ wis, const c2<T> *__restrict__ planes,
                                                 int log2nu, int log2nv, int Ww, T beta, T wbeta, int coplanar,
                                                 int taylor, const uint32_t *__restrict__ r_idx,
                                                 const uint32_t *__restrict__ r_cell, const T *__restrict__ r_du,
                                                 const T *__restrict__ r_dv, const T *__restrict__ r_dw,
                                                 const T *__restrict__ r_ph, const T *__restrict__ weight,
                                                 c2<T> *__restrict__ vis, int sorted_out,
                                                 const uint32_t *__restrict__ dpair) {
    static_assert(!PAIR || VPT == 2, "a pair is two records");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *tile = reinterpret_cast<c2<T> *>(smem_raw);
    constexpr int TS = kTile + W - 1;
    const WorkItem it = wis[blockIdx.x];
    const int nu = 1 << log2nu, nv = 1 << log2nv;
    const T two_over_W = T(2) / T(W);
    T ku[VPT][W], kv[VPT][W];
    T fw[VPT];
    int ru[VPT], rv[VPT];
    bool ok[VPT];
    int jrec[VPT];  // record of slot k inside the item
    c2<T> acc[VPT];
    if constexpr (PAIR) {
        // pair entry: first record | second record << 10 | alone << 20
        const bool act = (int)threadIdx.x < it.rows;
        const uint32_t e = act ? dpair[it.start + threadIdx.x] : 0u;
        jrec[0] = (int)(e & 1023u);
        jrec[1] = (int)((e >> 10) & 1023u);
        ok[0] = act;
        ok[1] = act && !((e >> 20) & 1u);
    } else {
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            jrec[k] = threadIdx.x + k * NTHR;
            ok[k] = jrec[k] < it.count;
        }
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int j = jrec[k];
        acc[k] = mk<T>(T(0), T(0));
        ru[k] = rv[k] = 0;
        fw[k] = T(0);
        // a lone record of a pair repeats the first one (interpolated, not stored)
        if (PAIR ? ok[0] : ok[k]) {
            const int64_t pos = it.start + j;
            const uint32_t c = r_cell[pos];
            ru[k] = (int)(c & 0xffffu);
            rv[k] = (int)(c >> 16);
            const T xu = r_du[pos], xv = r_dv[pos];
#pragma unroll
            for (int a = 0; a < W; ++a) {
                ku[k][a] = es_eval<T>((xu - T(a)) * two_over_W, beta);
                kv[k][a] = es_eval<T>((xv - T(a)) * two_over_W, beta);
            }
            fw[k] = r_dw[pos];
        }
    }
    // the tile of plane pw + 1 is fetched into registers while plane pw is used;
    // only the rows the item's footprints reach are staged (its records are sorted
    // by base cell: the first and the last hold the smallest and largest base row)
    const int q0 = (int)(r_cell[it.start] & 0xffffu) * TS;
    const int q1 = ((int)(r_cell[it.start + it.count - 1] & 0xffffu) + W) * TS;
    constexpr int NLD = (TS * TS + NTHR - 1) / NTHR;
    T pre_x[NLD], pre_y[NLD];
    int64_t toff[NLD];  // tile element offsets inside a plane
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int q = min(threadIdx.x + u * NTHR, TS * TS - 1);
        const int i = q / TS, jj = q - i * TS;
        toff[u] = ((int64_t)((it.tu + i) & (nu - 1)) << log2nv) + ((it.tv + jj) & (nv - 1));
    }
    auto fetch = [&](int p) {
        const c2<T> *P = planes + ((int64_t)p << (log2nu + log2nv));
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int q = threadIdx.x + u * NTHR;
            if (q >= q0 && q < q1) {
                const c2<T> g = P[toff[u]];
                pre_x[u] = g.x;
                pre_y[u] = g.y;
            }
        }
    };
    fetch(it.p0);
    for (int pw = 0; pw < Ww; ++pw) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int q = threadIdx.x + u * NTHR;
            if (q >= q0 && q < q1) tile[q] = mk<T>(pre_x[u], pre_y[u]);
        }
        __syncthreads();
        if (pw + 1 < Ww) fetch(it.p0 + pw + 1);
        if constexpr (PAIR) {
            // both records of the pair from the same tile reads (one base cell)
            if (ok[0]) {
                const T kw0 = coplanar ? T(1) : plane_weight<T>(fw[0], pw, Ww, wbeta, taylor);
                const T kw1 = coplanar ? T(1) : plane_weight<T>(fw[1], pw, Ww, wbeta, taylor);
                T sx0 = 0, sy0 = 0, sx1 = 0, sy1 = 0;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const c2<T> *rowp = tile + (ru[0] + a) * TS + rv[0];
                    T rx0 = 0, ry0 = 0, rx1 = 0, ry1 = 0;
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const c2<T> g = rowp[b];
                        rx0 += kv[0][b] * g.x;
                        ry0 += kv[0][b] * g.y;
                        rx1 += kv[1][b] * g.x;
                        ry1 += kv[1][b] * g.y;
                    }
                    sx0 += ku[0][a] * rx0;
                    sy0 += ku[0][a] * ry0;
                    sx1 += ku[1][a] * rx1;
                    sy1 += ku[1][a] * ry1;
                }
                acc[0].x += kw0 * sx0;
                acc[0].y += kw0 * sy0;
                acc[1].x += kw1 * sx1;
                acc[1].y += kw1 * sy1;
            }
        } else {
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                if (!ok[k]) continue;
                const T kw = coplanar ? T(1) : plane_weight<T>(fw[k], pw, Ww, wbeta, taylor);
                T sx = 0, sy = 0;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const c2<T> *rowp = tile + (ru[k] + a) * TS + rv[k];
                    T rx = 0, ry = 0;
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const c2<T> g = rowp[b];
                        rx += kv[k][b] * g.x;
                        ry += kv[k][b] * g.y;
                    }
                    sx += ku[k][a] * rx;
                    sy += ku[k][a] * ry;
                }
                acc[k].x += kw * sx;
                acc[k].y += kw * sy;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        if (!ok[k]) continue;
        const int64_t pos = it.start + jrec[k];
        c2<T> v = acc[k];
        if (sorted_out) {
            // w times the interpolated plane values in record order, for gridding
            // straight back (R^+ N^-1 R): the centring phase and the conjugation of
            // w < 0 records cancel between R and R^+
            if (weight) {
                const T wt = weight[r_idx[pos] & 0x7fffffffu];
                v.x *= wt;
                v.y *= wt;
            }
            vis[pos] = v;
            continue;
        }
        if (!coplanar) {
            T s, c;
            sincos_cycles(-r_ph[pos], &s, &c);
            v = cmul<T>(v, mk<T>(c, s));
        }
        const uint32_t id = r_idx[pos];
        if (id >> 31) v.y = -v.y;
        const uint32_t vi = id & 0x7fffffffu;
        if (weight) {  // N^-1 R: the diagonal noise weights applied in the store
            const T wt = weight[vi];
            v.x *= wt;
            v.y *= wt;
        }
        vis[vi] = v;
    }
}

// value of lane (byte_addr / 4) in each lane (ds_bpermute)
__device__ __forceinline__ float lane_permute(float v, int byte_addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
}
__device__ __forceinline__ double lane_permute(double v, int byte_addr) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(byte_addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value of lane k (wave-uniform k) in every lane
__device__ __forceinline__ float wave_bcast(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double wave_bcast(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ------------------------------------------------------------------ grid: partial tiles
// Planes held in registers per pass of the gridding kernel: lane (a, b) keeps,
// for each footprint cell it owns and each plane of the pass, the running sum of
// the current run of visibilities (about 48 VGPRs at most).
template <typename T, int W> constexpr int grid_reg_planes() {
    constexpr int ncell = (W * W + 63) / 64;
    constexpr int per_plane = ncell * 2 * (int)sizeof(T) / 4;
    return 48 / per_plane < 1 ? 1 : 48 / per_plane;
}

// One workgroup per gridding item (a chunk of the visibilities of one uv tile
// and first w-plane; the plan orders them by base cell inside the tile).  Each
// wavefront takes a contiguous share of the item in batches of 64: lane j loads
// record j and forms y_j times the w-kernel weight of every plane; the 1-D kernel
// values psi(du - a), psi(dv - a) are evaluated for 64 / W visibilities at a time
// (one lane per value).  The walk then takes one visibility at a time: lane
// (a, b) owns footprint cell (a, b) (cells beyond 64 wrap to more registers),
// fetches its psi pair with lane permutes and the plane values with readlane,
// and accumulates psi_u psi_v y psi_w per plane.  While consecutive visibilities
// share a base cell their contributions add up in registers; when the cell
// changes the run is flushed to the LDS tiles with one atomic per (cell, plane)
// and part.  The LDS tiles hold 64-bit fixed-point integers: every contribution
// to a component is at most bound = count * max(|Re y| + |Im y|) of the call
// (kernel values are <= 1), so scaling by 2^k with bound * 2^k < 2^61 keeps
// every partial sum in range, integer atomics (much faster than LDS float
// atomics) add them exactly, and the tile sums do not depend on the order in
// which waves flush.  `ppass` planes are done per pass (bounded by LDS and
// registers).  The accumulated tiles, halo included, are written with plain
// stores to the item's slot of the partial buffer [item][Ww][TS*TS] (complex);
// k_grid_assemble adds them up.  Tiles are stored in LDS as separate real and
// imaginary arrays.
template <typename T, int W, int NTHR>
__global__ __launch_bounds__(NTHR) void k_grid_partial(const WorkItem *__restrict__ wis,
                                                       const int32_t *__restrict__ seg, c2<T> *__restrict__ partial,
                                                       int Ww, int ppass, T beta, T wbeta, int coplanar,
                                                       int taylor, const uint32_t *__restrict__ r_cell,
                                                       const T *__restrict__ r_du, const T *__restrict__ r_dv,
                                                       const T *__restrict__ r_dw, const T *__restrict__ r_ph,
                                                       const c2<T> *__restrict__ y_rec,
                                                       const float *__restrict__ ybound_partials, int n_ybound,
                                                       int sorted_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    long long *tile = reinterpret_cast<long long *>(smem_raw);  // [ppass][2][TS * TS]
    constexpr int TS = kTile + W - 1;
    constexpr int TT = TS * TS;
    constexpr int NCELL = (W * W + 63) / 64;
    constexpr int NWAVE = NTHR / 64;
    constexpr int PR = grid_reg_planes<T, W>() < W ? grid_reg_planes<T, W>() : W;
    constexpr int VPB = 64 / W;  // visibilities per kernel-evaluation step
    // the tiles start at zero; a pass's band output clears the rows it reads, which
    // hold every cell the pass touched, so they are zero again for the next pass
    for (int q = threadIdx.x; q < min(ppass, PR) * 2 * TT; q += NTHR) tile[q] = 0;
    // fixed-point exponent from the bound on every contribution
    __shared__ float wmax[NWAVE];
    {
        float m = 0.0f;
        for (int q = threadIdx.x; q < n_ybound; q += NTHR) m = fmaxf(m, ybound_partials[q]);
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    }
    __syncthreads();
    float ymax = 0.0f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) ymax = fmaxf(ymax, wmax[q]);
    // the workgroup's items: consecutive items of about equal estimated cost,
    // each writing its own slot of the partials
    for (int item = seg[blockIdx.x]; item < seg[blockIdx.x + 1]; ++item) {
        const WorkItem it = wis[item];
        int kexp = 0;
        if (ymax > 0.0f && ymax <= 3.0e38f) {
            int e;
            frexp(2.0 * (double)ymax * (double)it.count, &e);  // bound < 2^(e-1)
            kexp = 62 - e;
        }
        c2<T> *out = partial + (int64_t)item * Ww * TT;
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loop control
        const T two_over_W = T(2) / T(W);
        int ca[NCELL], cb[NCELL], au[NCELL], av[NCELL];
#pragma unroll
        for (int q = 0; q < NCELL; ++q) {
            const int c = lane + 64 * q;
            ca[q] = c < W * W ? c / W : -1;
            cb[q] = c < W * W ? c - (c / W) * W : 0;
            au[q] = 4 * max(ca[q], 0);
            av[q] = 4 * cb[q];
        }
        // this wavefront's contiguous share of the item
        const int share = (it.count + NWAVE - 1) / NWAVE;
        const int v_begin = min(it.count, wave * share), v_end = min(it.count, v_begin + share);
        const int pp = min(ppass, PR);
        for (int g0 = 0; g0 < Ww; g0 += pp) {
            const int np = min(pp, Ww - g0);
            T acc_re[NCELL][PR], acc_im[NCELL][PR];
#pragma unroll
            for (int q = 0; q < NCELL; ++q)
#pragma unroll
                for (int p = 0; p < PR; ++p) acc_re[q][p] = acc_im[q][p] = T(0);
            int run_cell = -1;  // base cell of the run held in acc (wave-uniform)
            auto flush = [&]() {
                const int ru = run_cell & 0xffff, rv = run_cell >> 16;
#pragma unroll
                for (int q = 0; q < NCELL; ++q) {
                    if (ca[q] < 0) continue;
                    const int off = (ru + ca[q]) * TS + rv + cb[q];
#pragma unroll
                    for (int p = 0; p < PR; ++p) {
                        if (p >= np) break;
                        unsigned long long *tp = reinterpret_cast<unsigned long long *>(tile + 2 * p * TT);
                        const long long vr = (long long)rint(ldexp((double)acc_re[q][p], kexp));
                        const long long vi = (long long)rint(ldexp((double)acc_im[q][p], kexp));
                        atomicAdd(tp + off, (unsigned long long)vr);
                        atomicAdd(tp + TT + off, (unsigned long long)vi);
                        acc_re[q][p] = acc_im[q][p] = T(0);
                    }
                }
            };
            for (int b0 = v_begin; b0 < v_end; b0 += 64) {
                // lane k loads visibility b0 + k (one memory round trip per 64) and
                // forms its weighted value y and the w-kernel weight of every plane
                // of the pass; the walk below broadcasts them with readlane
                const int nb = min(64, v_end - b0);
                int l_cell = 0;
                T l_xu = T(0), l_xv = T(0);
                c2<T> l_y = mk<T>(T(0), T(0));
                T l_kw[PR];
#pragma unroll
                for (int p = 0; p < PR; ++p) l_kw[p] = T(p == 0 ? 1 : 0);
                if (lane < nb) {
                    const int64_t pos = it.start + b0 + lane;
                    l_cell = (int)r_cell[pos];
                    c2<T> y = y_rec[pos];  // weighted (w < 0: conjugated) value in record order
                    l_xu = r_du[pos];
                    l_xv = r_dv[pos];
                    if (!coplanar) {
                        if (!sorted_in) {
                            T sn, cs;
                            sincos_cycles(r_ph[pos], &sn, &cs);
                            y = cmul<T>(y, mk<T>(cs, sn));
                        }
                        const T xw = r_dw[pos];
#pragma unroll
                        for (int p = 0; p < PR; ++p)
                            l_kw[p] = p < np ? plane_weight<T>(xw, g0 + p, Ww, wbeta, taylor) : T(0);
                    }
                    l_y = y;
                }
                // the separable kernel values: lane v W + a (v < VPB, a < W) evaluates
                // psi(du - a) and psi(dv - a) of visibility k0 + v, and lane (a, b) of
                // the walk fetches its pair with two lane permutes
                for (int k0 = 0; k0 < nb; k0 += VPB) {
                    const int vv = lane / W, aa = lane - (lane / W) * W;
                    const int src = min(k0 + vv, 63);
                    const T xu_v = __shfl(l_xu, src, 64), xv_v = __shfl(l_xv, src, 64);
                    const T phu = es_eval<T>((xu_v - T(aa)) * two_over_W, beta);
                    const T phv = es_eval<T>((xv_v - T(aa)) * two_over_W, beta);
                    const int kend = min(k0 + VPB, nb);
                    // the permutes for visibility k + 1 are issued before the work on k
                    // (byte addresses: lane base + a of the value psi(d - a))
                    T nu_[NCELL], nv_[NCELL];
#pragma unroll
                    for (int q = 0; q < NCELL; ++q) {
                        nu_[q] = lane_permute(phu, au[q]);
                        nv_[q] = lane_permute(phv, av[q]);
                    }
                    for (int k = k0; k < kend; ++k) {
                        T cu_[NCELL], cv_[NCELL];
#pragma unroll
                        for (int q = 0; q < NCELL; ++q) {
                            cu_[q] = nu_[q];
                            cv_[q] = nv_[q];
                        }
                        if (k + 1 < kend) {
                            const int base1 = (k + 1 - k0) * W * 4;
#pragma unroll
                            for (int q = 0; q < NCELL; ++q) {
                                nu_[q] = lane_permute(phu, base1 + au[q]);
                                nv_[q] = lane_permute(phv, base1 + av[q]);
                            }
                        }
                        const int cell = __builtin_amdgcn_readlane(l_cell, k);
                        if (cell != run_cell) {
                            if (run_cell >= 0) flush();
                            run_cell = cell;
                        }
                        const T yx = wave_bcast(l_y.x, k), yy = wave_bcast(l_y.y, k);
                        T kw[PR];
#pragma unroll
                        for (int p = 0; p < PR; ++p) kw[p] = wave_bcast(l_kw[p], k);
                        // lanes beyond the footprint (ca < 0) accumulate values that
                        // are never flushed
#pragma unroll
                        for (int q = 0; q < NCELL; ++q) {
                            const T w = cu_[q] * cv_[q];
                            const T wr = w * yx, wi = w * yy;
#pragma unroll
                            for (int p = 0; p < PR; ++p) {
                                acc_re[q][p] += wr * kw[p];
                                acc_im[q][p] += wi * kw[p];
                            }
                        }
                    }
                }
            }
            if (run_cell >= 0) flush();
            __syncthreads();
            // only the rows the item touched are stored (the assembly reads no others)
            const int r0 = it.rows & 0xffff, r1 = it.rows >> 16;
            const int band = (r1 - r0 + 1) * TS;
            for (int q = threadIdx.x; q < np * band; q += NTHR) {
                const int p = q / band, r = r0 * TS + (q - p * band);
                out[(int64_t)(g0 + p) * TT + r] = mk<T>((T)ldexp((double)tile[2 * p * TT + r], -kexp),
                                                        (T)ldexp((double)tile[2 * p * TT + TT + r], -kexp));
                tile[2 * p * TT + r] = 0;
                tile[2 * p * TT + TT + r] = 0;
            }
            __syncthreads();
        }
    }
}

// The same spread on the matrix cores (FP32, W <= 8, at most 8 planes per pass).
// Within a run of equal base cells the register sums are a dense contraction,
//   S[cell][n] = sum_k A[cell][k] B[k][n],
//   A[cell][k] = psi(du_k - a) psi(dv_k - b)   (cell = a W + b, 64 rows in 4 blocks of 16),
//   B[k][n]    = y_k times the plane-(n/2) weight of visibility k, real part for even
//                n and imaginary for odd (n < 16),
// taken four visibilities at a time with v_mfma_f32_16x16x4_f32 per block of 16
// cells.  Operand layout of that instruction (checked on the hardware): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16],
// r < 4.  The 1-D kernel values of 8 visibilities are evaluated at a time (lane
// 8 v + a holds psi(d_v - a)), as are the plane weights, and A and B are gathered
// from them with lane permutes once per group; visibilities outside the current
// run segment get B = 0.  Runs, flushes to the 64-bit fixed-point LDS tiles and
// the band output are as in k_grid_partial.
template <int W, int NTHR>
__global__ __launch_bounds__(NTHR) void k_grid_partial_mfma(
    const WorkItem *__restrict__ wis, const int32_t *__restrict__ seg, c2<float> *__restrict__ partial, int Ww,
    int ppass, float beta, float wbeta,
    int coplanar, int taylor, const uint32_t *__restrict__ r_cell,
    const float *__restrict__ r_du, const float *__restrict__ r_dv, const float *__restrict__ r_dw,
    const float *__restrict__ r_ph, const c2<float> *__restrict__ y_rec,
    const float *__restrict__ ybound_partials, int n_ybound, int sorted_in) {
    static_assert(W <= 8, "one lane per 1-D kernel value of 8 visibilities");
    typedef float v4f __attribute__((ext_vector_type(4)));
    extern __shared__ __align__(16) unsigned char smem_raw[];
    long long *tile = reinterpret_cast<long long *>(smem_raw);  // [ppass][2][TS * TS]
    constexpr int TS = kTile + W - 1;
    constexpr int TT = TS * TS;
    constexpr int NWAVE = NTHR / 64;
    constexpr int NBLK = (W * W + 15) / 16;  // blocks of 16 cells
    // the tiles start at zero; a pass's band output clears the rows it reads, which
    // hold every cell the pass touched, so they are zero again for the next pass
    for (int q = threadIdx.x; q < min(ppass, 8) * 2 * TT; q += NTHR) tile[q] = 0;
    __shared__ float wmax[NWAVE];
    {
        float m = 0.0f;
        for (int q = threadIdx.x; q < n_ybound; q += NTHR) m = fmaxf(m, ybound_partials[q]);
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    }
    __syncthreads();
    float ymax = 0.0f;
#pragma unroll
    for (int q = 0; q < NWAVE; ++q) ymax = fmaxf(ymax, wmax[q]);
    // the workgroup's items: consecutive items of about equal estimated cost,
    // each writing its own slot of the partials
    for (int item = seg[blockIdx.x]; item < seg[blockIdx.x + 1]; ++item) {
        const WorkItem it = wis[item];
        int kexp = 0;
        if (ymax > 0.0f && ymax <= 3.0e38f) {
            int e;
            frexp(2.0 * (double)ymax * (double)it.count, &e);  // bound < 2^(e-1)
            kexp = 62 - e;
        }
        c2<float> *out = partial + (int64_t)item * Ww * TT;
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const float two_over_W = 2.0f / (float)W;
        // A operand: row (cell) lane % 16 of each block, column (visibility) lane / 16
        const int kk = lane >> 4;
        int a_addr[NBLK], b_addr[NBLK];
#pragma unroll
        for (int blk = 0; blk < NBLK; ++blk) {
            const int c = 16 * blk + (lane & 15);
            const bool ok = c < W * W;
            const int ca = ok ? c / W : 0, cb = ok ? c - (c / W) * W : 0;
            a_addr[blk] = 4 * ca;  // byte offset of psi(du - a) inside a visibility's 8 lanes
            b_addr[blk] = 4 * cb;
        }
        // B operand: column n = lane % 16 -> plane n / 2, real or imaginary part
        const int n_col = lane & 15, p_col = n_col >> 1, im_col = n_col & 1;
        // D: lane holds cells 16 blk + 4 (lane / 16) + r of column n_col
        const int share = (it.count + NWAVE - 1) / NWAVE;
        const int v_begin = min(it.count, wave * share), v_end = min(it.count, v_begin + share);
        const int pp = min(ppass, 8);
        for (int g0 = 0; g0 < Ww; g0 += pp) {
            const int np = min(pp, Ww - g0);
            v4f acc[NBLK];
#pragma unroll
            for (int blk = 0; blk < NBLK; ++blk) acc[blk] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            int run_cell = -1;
            auto flush = [&]() {
                const int ru = run_cell & 0xffff, rv = run_cell >> 16;
                if (p_col < np) {
                    long long *tp = tile + (2 * p_col + im_col) * TT;
#pragma unroll
                    for (int blk = 0; blk < NBLK; ++blk)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int c = 16 * blk + 4 * kk + r;
                            if (c < W * W) {
                                const int ca = c / W, cb = c - (c / W) * W;
                                const long long v = (long long)rint(ldexp((double)acc[blk][r], kexp));
                                atomicAdd(reinterpret_cast<unsigned long long *>(tp + (ru + ca) * TS + rv + cb),
                                          (unsigned long long)v);
                            }
                        }
                }
#pragma unroll
                for (int blk = 0; blk < NBLK; ++blk) acc[blk] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            };
            for (int b0 = v_begin; b0 < v_end; b0 += 64) {
                const int nb = min(64, v_end - b0);
                int l_cell = 0;
                float l_xu = 0.0f, l_xv = 0.0f, l_xw = 0.0f;
                c2<float> l_y = mk<float>(0.0f, 0.0f);
                if (lane < nb) {
                    const int64_t pos = it.start + b0 + lane;
                    l_cell = (int)r_cell[pos];
                    c2<float> y = y_rec[pos];  // weighted (w < 0: conjugated) value in record order
                    l_xu = r_du[pos];
                    l_xv = r_dv[pos];
                    if (!coplanar) {
                        if (!sorted_in) {
                            float sn, cs;
                            sincos_cycles(r_ph[pos], &sn, &cs);
                            y = cmul<float>(y, mk<float>(cs, sn));
                        }
                        l_xw = r_dw[pos];
                    }
                    l_y = y;
                }
                // records that start a run (base cell differs from the previous record's)
                const int prev_cell = __shfl(l_cell, lane > 0 ? lane - 1 : 0, 64);
                const unsigned long long starts = __ballot(lane < nb && (lane == 0 || l_cell != prev_cell));
                for (int k0 = 0; k0 < nb; k0 += 8) {
                    // 1-D kernel values of visibilities k0 .. k0 + 7: lane 8 v + a
                    const int src = min(k0 + (lane >> 3), 63), ta = lane & 7;
                    const float xu_v = __shfl(l_xu, src, 64), xv_v = __shfl(l_xv, src, 64);
                    const float phu = ta < W ? es_eval<float>((xu_v - (float)ta) * two_over_W, beta) : 0.0f;
                    const float phv = ta < W ? es_eval<float>((xv_v - (float)ta) * two_over_W, beta) : 0.0f;
                    // plane weights of the same visibilities: lane 8 v + a holds plane g0 + a
                    float phw = 1.0f;
                    if (!coplanar) {
                        const float xw_v = __shfl(l_xw, src, 64);
                        phw = ta < np ? plane_weight<float>(xw_v, g0 + ta, Ww, wbeta, taylor) : 0.0f;
                    }
                    // operands of both halves of the group, gathered once for all its
                    // run segments (lanes outside a segment get B = 0).  All lane
                    // permutes are issued before the first product, so their latency
                    // is paid once per group rather than once per block.
                    float ua[2][NBLK], va[2][NBLK], kwa[2], yxa[2], yya[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int q = k0 + 4 * s + kk;  // this lane's visibility in A and B
                        const int sq = min(q, 63);
                        const int vbase = 32 * (4 * s + kk);  // byte offset of visibility q's 8 lanes
                        yxa[s] = __shfl(l_y.x, sq, 64);
                        yya[s] = __shfl(l_y.y, sq, 64);
                        kwa[s] = lane_permute(phw, vbase + 4 * p_col);
#pragma unroll
                        for (int blk = 0; blk < NBLK; ++blk) {
                            ua[s][blk] = lane_permute(phu, vbase + a_addr[blk]);
                            va[s][blk] = lane_permute(phv, vbase + b_addr[blk]);
                        }
                    }
                    // A: psi(du_q - a) psi(dv_q - b) of the lane's cell in each block
                    // (finite everywhere; rows of cells beyond W^2 are never flushed);
                    // B before the segment mask: y_q times its plane-(g0 + p_col) weight
                    float aop[2][NBLK], bop[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        bop[s] = kwa[s] * (im_col ? yya[s] : yxa[s]);
#pragma unroll
                        for (int blk = 0; blk < NBLK; ++blk) aop[s][blk] = ua[s][blk] * va[s][blk];
                    }
                    const int kend = min(k0 + 8, nb);
                    int k = k0;
                    while (k < kend) {
                        // the run segment [k, ke) of equal base cells inside this group
                        const int cell = __builtin_amdgcn_readlane(l_cell, k);
                        if (cell != run_cell) {
                            if (run_cell >= 0) flush();
                            run_cell = cell;
                        }
                        // the segment ends at the next run start inside the group
                        // (shift counts stay below 64: k < kend <= 64)
                        const unsigned long long above = (k >= 63) ? 0ull : (~0ull << (k + 1));
                        const unsigned long long below = (kend >= 64) ? ~0ull : ((1ull << kend) - 1ull);
                        const unsigned long long later = starts & above & below;
                        const int ke = later ? __builtin_ctzll(later) : kend;  // k < ke <= kend
#pragma unroll
                        for (int s = 0; s < 2; ++s) {
                            // a half the segment does not reach has B = 0 in every lane:
                            // its products would add exact zeros, so they are not issued
                            if (ke <= k0 + 4 * s || k >= k0 + 4 * s + 4) continue;
                            // B is zero outside the segment, which also cancels A there
                            const int q = k0 + 4 * s + kk;
                            const bool use = q >= k && q < ke && p_col < np;
                            const float bval = use ? bop[s] : 0.0f;
#pragma unroll
                            for (int blk = 0; blk < NBLK; ++blk)
                                acc[blk] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[s][blk], bval, acc[blk], 0, 0, 0);
                        }
                        k = ke;
                    }
                }
            }
            if (run_cell >= 0) flush();
            __syncthreads();
            const int r0 = it.rows & 0xffff, r1 = it.rows >> 16;
            const int band = (r1 - r0 + 1) * TS;
            for (int q = threadIdx.x; q < np * band; q += NTHR) {
                const int p = q / band, r = r0 * TS + (q - p * band);
                out[(int64_t)(g0 + p) * TT + r] = mk<float>((float)ldexp((double)tile[2 * p * TT + r], -kexp),
                                                            (float)ldexp((double)tile[2 * p * TT + TT + r], -kexp));
                tile[2 * p * TT + r] = 0;
                tile[2 * p * TT + TT + r] = 0;
            }
            __syncthreads();
        }
    }
}

// partials[b] = block b's maximum over visibilities of (|Re v| + |Im v|) |w|
// (v = 1 without visibilities, w = 1 without weights), rounded up to FP32
template <typename T>
__global__ __launch_bounds__(256) void k_vis_bound(const c2<T> *__restrict__ vis, const T *__restrict__ weight,
                                                   int64_t n, float *__restrict__ partials) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double a = 1.0;
        if (vis) a = fabs((double)vis[i].x) + fabs((double)vis[i].y);
        if (weight) a *= fabs((double)weight[i]);
        m = fmaxf(m, __double2float_ru(a));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

// The same bound, and the weighted values y = w v (v = 1 without visibilities,
// conjugated for records folded from w < 0) scattered into record order through
// the plan's record positions, so that the spread reads them with coalesced
// loads instead of gathering each record's visibility and weight by its
// original index.  The centring phase stays with the spread.
template <typename T>
__global__ __launch_bounds__(256) void k_vis_prepare(const c2<T> *__restrict__ vis, const T *__restrict__ weight,
                                                     const uint32_t *__restrict__ r_pos, int64_t n,
                                                     float *__restrict__ partials, c2<T> *__restrict__ y_rec) {
    // four values per thread and pass, their loads issued before any store
    constexpr int U = 4;
    float m = 0.0f;
    for (int64_t base = (int64_t)blockIdx.x * 256 * U + threadIdx.x; base < n; base += (int64_t)gridDim.x * 256 * U) {
        c2<T> y[U];
        T wt[U];
        uint32_t ps[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + u * 256;
            if (i < n) {
                y[u] = vis ? vis[i] : mk<T>(T(1), T(0));
                wt[u] = weight ? weight[i] : T(1);
                ps[u] = r_pos[i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * 256 >= n) break;
            c2<T> v = y[u];
            double a = fabs((double)v.x) + fabs((double)v.y);
            if (weight) {
                a *= fabs((double)wt[u]);
                v.x *= wt[u];
                v.y *= wt[u];
            }
            m = fmaxf(m, __double2float_ru(a));
            if (ps[u] >> 31) v.y = -v.y;
            y_rec[ps[u] & 0x7fffffffu] = v;
        }
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    __shared__ float sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

// Owner-computes assembly: workgroup (active tile, plane p) writes the 32 x 32
// cells it owns, one per thread, each the sum, in a fixed order, of the partial tiles that
// cover it: the items of its own tile and of the tiles up to one step back in u
// and v (their W - 1 halo reaches into this tile), for every first plane p0 with
// p - Ww < p0 <= p.  The items of a tile are sorted by base cell, so those that
// touch a given tile row form a contiguous run, found by binary search on their
// first and last rows (once per workgroup, into LDS).  Every cell of an active
// tile is written exactly once;
// the inverse column transform reads zeros for the other tiles, so the planes
// need no clearing and the result does not depend on scheduling.  Eight partial
// loads are kept in flight per thread.
template <typename T, int W>
__global__ __launch_bounds__(kTile * kTile) void k_grid_assemble(const c2<T> *__restrict__ partial,
                                                                 const int32_t *__restrict__ atile,
                                                                 const WorkItem *__restrict__ items,
                                                                 const uint32_t *__restrict__ gkey_first,
                                                                 int64_t item0, int64_t key0, int n_p0, int ntu,
                                                                 int ntv, int Ww, int log2nu, int log2nv,
                                                                 c2<T> *__restrict__ planes) {
    constexpr int TS = kTile + W - 1;
    constexpr int TT = TS * TS;
    constexpr int U = 8;
    const int t = atile[blockIdx.x];
    const int p = blockIdx.y;
    const int tu = t / ntv, tv = t - tu * ntv;
    const int n_tiles = ntu * ntv;
    const int pmin = max(0, p - Ww + 1), pmax = min(p, n_p0 - 1);
    const int64_t stride = (int64_t)Ww * TT;  // between consecutive items
    // item ranges per (column step dj, first plane p0, tile row li), found once per
    // workgroup by parallel binary searches: items of a key are sorted by rows, so
    // those touching row li are [first whose last row reaches li, first whose
    // first row passes li)
    const int np = pmax - pmin + 1;
    __shared__ uint2 range[2 * W * TS];
    for (int q = threadIdx.x; q < 2 * np * TS; q += kTile * kTile) {
        const int li = q % TS, r = q / TS;
        const int dj = r / np, p0 = pmin + (r - dj * np);
        const int di = li >= kTile ? 1 : 0;
        const int t2 = ((tu - di + ntu) % ntu) * ntv + (tv - dj + ntv) % ntv;
        const int64_t key = key0 + (int64_t)p0 * n_tiles + t2;
        const uint32_t b = gkey_first[key], e = gkey_first[key + 1];
        uint32_t lo = b, hi = e;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((items[mid].rows >> 16) < li) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t first = lo;
        hi = e;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((items[mid].rows & 0xffff) <= li) lo = mid + 1;
            else hi = mid;
        }
        range[q] = make_uint2(first, lo);
    }
    __syncthreads();
    const int i = threadIdx.x / kTile, j = threadIdx.x - (threadIdx.x / kTile) * kTile;
    T sx = 0, sy = 0;
    for (int di = 0; di < 2; ++di) {
        const int li = i + di * kTile;
        if (li >= TS) continue;
        for (int dj = 0; dj < 2; ++dj) {
            const int lj = j + dj * kTile;
            if (lj >= TS) continue;
            for (int p0 = pmin; p0 <= pmax; ++p0) {
                const uint2 rg = range[(dj * np + (p0 - pmin)) * TS + li];
                const uint32_t b = rg.x, e = rg.y;
                const c2<T> *src = partial + ((int64_t)(b - item0) * Ww + (p - p0)) * TT + li * TS + lj;
                const uint32_t n = e - b;
                uint32_t k = 0;
                for (; k + U <= n; k += U) {
                    c2<T> v[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) v[u] = src[(int64_t)(k + u) * stride];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        sx += v[u].x;
                        sy += v[u].y;
                    }
                }
                for (; k < n; ++k) {
                    const c2<T> v = src[(int64_t)k * stride];
                    sx += v.x;
                    sy += v.y;
                }
            }
        }
    }
    const int a = tu * kTile + i, b2 = tv * kTile + j;
    planes[((((int64_t)p << log2nu) + a) << log2nv) + b2] = mk<T>(sx, sy);
}

// ------------------------------------------------------------------ FFT functors
// row transform of degridding: line = p * nx + i
// (image sides are powers of two: line = p nx + i splits with shifts)
template <typename T> struct DegridRowPro {
    const T *img, *fac, *tpix;  // tpix: Taylor variable tau per pixel (Taylor plans)
    const double *tpix_w;       // (n - 1) - yc per pixel (w-stacked plans)
    const double *wplane;
    int nx, ny, nv, coplanar, taylor;
    __device__ c2<T> operator()(int64_t line, int b) const {
        const int p = (int)line >> (31 - __builtin_clz(nx));
        const int i = (int)line & (nx - 1);
        const int j = (b + ny / 2) & (nv - 1);
        if (j >= ny) return mk<T>(T(0), T(0));
        const int64_t q = (int64_t)i * ny + j;
        const T f = img[q] * fac[q];
        if (coplanar) return mk<T>(f, T(0));
        if (taylor) {
            // Taylor term p: f (-i tau)^p with tau = ((n - 1) - yc) / h
            T g = f;
            for (int k = 0; k < p; ++k) g *= tpix[q];
            switch (p & 3) {
                case 0: return mk<T>(g, T(0));
                case 1: return mk<T>(T(0), -g);
                case 2: return mk<T>(-g, T(0));
                default: return mk<T>(T(0), g);
            }
        }
        // the plane phase w_p t in cycles, reduced modulo 1 in double before rounding
        double ph = wplane[p] * tpix_w[q];
        ph -= rint(ph);
        T s, c;
        sincos_cycles(-(T)ph, &s, &c);
        return mk<T>(f * c, f * s);
    }
};
template <typename T> struct DegridRowEpi {
    c2<T> *planes;
    const uint8_t *col_active;  // [ntv] of the channel: columns no degridding reads are not stored
    int nx, log2nu, log2nv;
    __device__ void operator()(int64_t line, int b, c2<T> v) const {
        if (!col_active[b / kTile]) return;
        const int p = (int)line >> (31 - __builtin_clz(nx));
        const int i = (int)line & (nx - 1);
        const int a = (i - nx / 2) & ((1 << log2nu) - 1);
        planes[((((int64_t)p << log2nu) + a) << log2nv) + b] = v;
    }
};
// column access of plane m; rows outside the image band are zero (never read)
template <typename T> struct BandColPro {
    const c2<T> *planes;
    int nx, log2nu, log2nv;
    __device__ c2<T> operator()(int64_t m, int a, int b) const {
        const int nu = 1 << log2nu;
        if (a >= nx / 2 && a < nu - nx / 2) return mk<T>(T(0), T(0));
        return planes[(((m << log2nu) + a) << log2nv) + b];
    }
};
template <typename T> struct FullColPro {
    const c2<T> *planes;
    int log2nu, log2nv;
    __device__ c2<T> operator()(int64_t m, int a, int b) const { return planes[(((m << log2nu) + a) << log2nv) + b]; }
};
// gridded planes: tiles without active flag are zero and not read
template <typename T> struct ActiveColPro {
    const c2<T> *planes;
    const uint8_t *active;  // [n_tiles] of the channel
    int log2nu, log2nv, ntv;
    __device__ c2<T> operator()(int64_t m, int a, int b) const {
        if (!active[(a / kTile) * ntv + b / kTile]) return mk<T>(T(0), T(0));
        return planes[(((m << log2nu) + a) << log2nv) + b];
    }
};
template <typename T> struct FullColEpi {
    c2<T> *planes;
    int log2nu, log2nv;
    __device__ void operator()(int64_t m, int a, int b, c2<T> v) const {
        planes[(((m << log2nu) + a) << log2nv) + b] = v;
    }
};
// stores only the cells of active tiles (the only ones degridding reads)
template <typename T> struct ActiveColEpi {
    c2<T> *planes;
    const uint8_t *active;  // [n_tiles] of the channel
    int log2nu, log2nv, ntv;
    __device__ void operator()(int64_t m, int a, int b, c2<T> v) const {
        if (!active[(a / kTile) * ntv + b / kTile]) return;
        planes[(((m << log2nu) + a) << log2nv) + b] = v;
    }
};
template <typename T> struct BandColEpi {
    c2<T> *planes;
    int nx, log2nu, log2nv;
    __device__ void operator()(int64_t m, int a, int b, c2<T> v) const {
        const int nu = 1 << log2nu;
        if (a >= nx / 2 && a < nu - nx / 2) return;
        planes[(((m << log2nu) + a) << log2nv) + b] = v;
    }
};

// Gridding epilogue: image row i accumulates Re(exp(+2 pi i w_p t) G_p) over planes,
// transforming `lines` plane rows at a time (all threads busy in every stage).
template <typename T, int NTHR, int BPT, int ACC, bool TWL>
__global__ __launch_bounds__(NTHR) void k_grid_rows(const c2<T> *__restrict__ planes,
                                                    const uint8_t *__restrict__ col_active, int n_planes, int log2nu,
                                                    int log2nv, int nx, int ny, const T *__restrict__ fac,
                                                    const T *__restrict__ tpix, const double *__restrict__ tpix_w,
                                                    const double *__restrict__ wplane,
                                                    int coplanar, int taylor, T *__restrict__ img, int lines,
                                                    const c2<T> *__restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int i = blockIdx.x;
    const int nu = 1 << log2nu, nv = 1 << log2nv;
    const int ld = plen(nv);
    const int a = (i - nx / 2) & (nu - 1);
    T acc[ACC];
#pragma unroll
    for (int k = 0; k < ACC; ++k) acc[k] = T(0);
    // the row loads of this thread touch columns (threadIdx.x + j NTHR) mod nv,
    // j < J: which of them lie in a tile column holding an active tile (the others
    // are zero in every plane and not stored), as a bit mask
    const int J = nv > NTHR ? nv / NTHR : 1;  // at most 64 (host-checked)
    unsigned long long cmask = 0;
    for (int j = 0; j < J; ++j)
        if (col_active[((threadIdx.x + j * NTHR) & (nv - 1)) / kTile]) cmask |= 1ull << j;
    constexpr int LOG2N = __builtin_ctz(NTHR);
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + lines * ld, tw, nv);
    for (int p0 = 0; p0 < n_planes; p0 += lines) {
        const int nl = min(lines, n_planes - p0);
        staged_copy<NTHR>(
            nl << log2nv,
            [&](int idx) {
                // idx = threadIdx.x + k NTHR: column (threadIdx.x + (k mod J) NTHR) mod nv
                if (!((cmask >> ((idx >> LOG2N) & (J - 1))) & 1ull)) return mk<T>(T(0), T(0));
                const int64_t row = ((int64_t)(p0 + (idx >> log2nv)) << log2nu) + a;
                return planes[(row << log2nv) + (idx & (nv - 1))];
            },
            [&](int idx, c2<T> v) { buf[(idx >> log2nv) * ld + padx(idx & (nv - 1))] = v; });
        __syncthreads();
        // compile-time stages for rows of 512 and 1024 points only (the 1024-thread
        // form runs rows of 8192 points and more): this kernel is short of registers
        lds_fft<T, NTHR, BPT, 1, (NTHR < 1024 ? 0x600u : 0u)>(buf, ld, nl, log2nv, +1, twp);
        for (int l = 0; l < nl; ++l) {
            const double wp = wplane[p0 + l];
            const c2<T> *line = buf + l * ld;
#pragma unroll
            for (int k = 0; k < ACC; ++k) {
                const int j = threadIdx.x + k * NTHR;
                if (j < ny) {
                    const c2<T> g = line[padx((j - ny / 2) & (nv - 1))];
                    if (coplanar) {
                        acc[k] += g.x;
                    } else if (taylor) {
                        // adjoint of term p: tau^p Re(i^p G)
                        const int p = p0 + l;
                        T tp = T(1);
                        for (int e = 0; e < p; ++e) tp *= tpix[(int64_t)i * ny + j];
                        const T re = (p & 1) ? ((p & 2) ? g.y : -g.y) : ((p & 2) ? -g.x : g.x);
                        acc[k] += tp * re;
                    } else {
                        double ph = wp * tpix_w[(int64_t)i * ny + j];
                        ph -= rint(ph);
                        T s, c;
                        sincos_cycles((T)ph, &s, &c);
                        acc[k] += g.x * c - g.y * s;
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < ACC; ++k) {
        const int j = threadIdx.x + k * NTHR;
        if (j < ny) img[(int64_t)i * ny + j] = fac[(int64_t)i * ny + j] * acc[k];
    }
}

template <typename T> __global__ void k_zero(T *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

template <typename T> void zero_async(T *p, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    ProfScope prof("zero", st);
    k_zero<T><<<dim3((unsigned)blocks), 256, 0, st>>>(p, n);
    LAUNCH_CHECK();
}

// ------------------------------------------------------------------ launch helpers
// Records per degridding item, one thread each (FP32: 512 threads measured 6%
// faster than 256 threads with two records each, the registers per thread
// dropping enough for more resident waves).
template <typename T> constexpr int chunk() { return std::is_same<T, float>::value ? 512 : 256; }
// pair-list entries per paired degridding item (one per thread)
constexpr int kPairsPerItem = 256;

template <typename T, int W>
void launch_degrid_w(const fr_plan *pl, const WorkItem *wis, int64_t nwi, const c2<T> *planes, const T *weight,
                     c2<T> *vis, hipStream_t st, int sorted_out) {
    constexpr int TS = kTile + W - 1;
    const size_t lds = (size_t)TS * TS * sizeof(c2<T>);
    ProfScope prof("degrid", st);
    auto launch = [&](auto kern, int nthr) {
        allow_lds(kern, lds);
        kern<<<dim3((unsigned)nwi), nthr, lds, st>>>(
            wis, planes, ilog2(pl->nu), ilog2(pl->nv), pl->Ww, (T)pl->beta, (T)pl->wbeta, pl->coplanar ? 1 : 0,
            pl->taylor ? 1 : 0, pl->r_idx.as<uint32_t>(), pl->r_cell.as<uint32_t>(), pl->r_du.as<T>(),
            pl->r_dv.as<T>(), pl->r_dw.as<T>(), pl->r_ph.as<T>(), weight, vis, sorted_out, pl->dpair.as<uint32_t>());
    };
    // runs of several records: two records of a base cell per thread share the tile
    // reads; the plan cuts paired items at kPairsPerItem entries (and chunk records)
    bool done = false;
    if constexpr (std::is_same<T, float>::value) {
        if (paired_degrid(pl)) {
            launch(k_degrid<T, W, kPairsPerItem, 2, true>, kPairsPerItem);
            done = true;
        }
    }
    if (!done) launch(k_degrid<T, W, chunk<T>(), 1, false>, chunk<T>());
    LAUNCH_CHECK();
}

// Launch shape of the gridding spread: threads per workgroup (FP64 and wide
// kernels hold more registers per lane: smaller groups, larger register share),
// planes per pass and LDS bytes (one float per wavefront is static), and how many
// of its workgroups one CU holds.
struct GridShape {
    int nthr, ppass, per_cu;
    size_t lds;
};
static GridShape grid_shape(int W, int Ww, bool fp64) {
    GridShape g;
    g.nthr = (fp64 || W * W > 64) ? 512 : 1024;
    const size_t TS = kTile + W - 1;
    const size_t per_plane_lds = TS * TS * 2 * sizeof(long long);
    const size_t lds_static = (size_t)(g.nthr / 64) * sizeof(float);
    const size_t lds_dyn = (size_t)kLdsBytes - lds_static;
    g.ppass = (int)std::max<size_t>(1, std::min<size_t>((size_t)Ww, lds_dyn / per_plane_lds));
    g.lds = per_plane_lds * g.ppass;
    g.per_cu = (int)std::max<size_t>(1, std::min<size_t>((size_t)kLdsBytes / (g.lds + lds_static), 2048 / g.nthr));
    return g;
}

// Records per gridding workgroup at least (channels of fewer records per CU use
// fewer workgroups, so that they write few partial tiles).
constexpr int64_t kMinRangeRecords = 2048;

template <typename T, int W>
void launch_grid_w(const fr_plan *pl, int64_t chan, c2<T> *planes, const c2<T> *y_rec, const float *ybound,
                   int nbb, hipStream_t st, int sorted_in) {
    constexpr int TS = kTile + W - 1;
    constexpr int NTHR = (sizeof(T) == 8 || W * W > 64) ? 512 : 1024;
    const int64_t i0 = pl->gwi_chan[chan], i1 = pl->gwi_chan[chan + 1];
    const size_t per_plane = (size_t)TS * TS * sizeof(c2<T>);
    const GridShape gs = grid_shape(W, pl->Ww, sizeof(T) == 8);
    FR_REQUIRE(gs.nthr == NTHR, "gridding launch shape");
    if (i1 > i0) {
        // the channel's workgroups, each taking a range of its items
        const int64_t s0 = pl->gseg_chan[chan], n_wg = pl->gseg_chan[chan + 1] - s0 - 1;
        Scratch partial((size_t)(i1 - i0) * pl->Ww * per_plane, st);
        const int ppass = gs.ppass;
        const size_t lds = gs.lds;
        {
            ProfScope prof("grid", st);
            auto launch_vector = [&]() {
                auto kern = k_grid_partial<T, W, NTHR>;
                allow_lds(kern, lds);
                kern<<<dim3((unsigned)n_wg), NTHR, lds, st>>>(
                    pl->gwi.as<WorkItem>() + i0, pl->gseg.as<int32_t>() + s0, partial.as<c2<T>>(), pl->Ww, ppass,
                    (T)pl->beta, (T)pl->wbeta, pl->coplanar ? 1 : 0, pl->taylor ? 1 : 0,
                    pl->r_cell.as<uint32_t>(), pl->r_du.as<T>(), pl->r_dv.as<T>(), pl->r_dw.as<T>(), pl->r_ph.as<T>(),
                    y_rec, ybound, nbb, sorted_in);
            };
            if constexpr (std::is_same<T, float>::value && W <= 8) {
                // FP32, footprint <= 64 cells and runs of several records (an MFMA
                // step takes 4 records of one run; measured 1.4x faster than the
                // vector kernel at 62 records per run, 1.5x slower at ~1): the run
                // sums on the matrix cores
                if (matrix_spread(pl)) {
                    auto kern = k_grid_partial_mfma<W, NTHR>;
                    allow_lds(kern, lds);
                    kern<<<dim3((unsigned)n_wg), NTHR, lds, st>>>(
                        pl->gwi.as<WorkItem>() + i0, pl->gseg.as<int32_t>() + s0, partial.as<c2<T>>(), pl->Ww,
                        ppass, (T)pl->beta, (T)pl->wbeta, pl->coplanar ? 1 : 0, pl->taylor ? 1 : 0,
                        pl->r_cell.as<uint32_t>(), pl->r_du.as<T>(), pl->r_dv.as<T>(),
                        pl->r_dw.as<T>(), pl->r_ph.as<T>(), y_rec, ybound, nbb, sorted_in);
                } else {
                    launch_vector();
                }
            } else {
                launch_vector();
            }
            LAUNCH_CHECK();
        }
        ProfScope prof("grid_assemble", st);
        const int64_t a0 = pl->atile_chan[chan], a1 = pl->atile_chan[chan + 1];
        k_grid_assemble<T, W><<<dim3((unsigned)(a1 - a0), (unsigned)pl->n_planes), kTile * kTile, 0, st>>>(
            partial.as<c2<T>>(), pl->atile.as<int32_t>() + a0, pl->gwi.as<WorkItem>(), pl->gkey_first.as<uint32_t>(), i0,
            chan * pl->n_p0 * (int64_t)pl->n_tiles,
            pl->n_p0, pl->ntu, pl->ntv, pl->Ww, ilog2(pl->nu), ilog2(pl->nv), planes);
        LAUNCH_CHECK();
    }
    // a channel without visibilities has no active tile: its planes are never read
}

#define FR_W_DISPATCH(W_, CALL) \
    switch (W_) {               \
    case 4: CALL(4); break;     \
    case 5: CALL(5); break;     \
    case 6: CALL(6); break;     \
    case 7: CALL(7); break;     \
    case 8: CALL(8); break;     \
    case 9: CALL(9); break;     \
    case 10: CALL(10); break;   \
    case 11: CALL(11); break;   \
    case 12: CALL(12); break;   \
    case 13: CALL(13); break;   \
    case 14: CALL(14); break;   \
    case 15: CALL(15); break;   \
    case 16: CALL(16); break;   \
    default: throw Error(FR_EINVAL, "unsupported kernel support"); \
    }

size_t planes_bytes(const fr_plan *pl) {
    return (size_t)pl->n_planes * pl->nu * pl->nv * (pl->fp64 ? sizeof(double2) : sizeof(float2));
}

// Blocks of k_vis_bound (one partial maximum each).
static int vis_bound_blocks(int64_t n_vis) {
    return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n_vis + 1023) / 1024));
}

// Partial tiles of the largest channel: [items][Ww][TS * TS] complex.
static size_t grid_partial_bytes(int64_t items, int Ww, int W, bool fp64) {
    const size_t TS = kTile + W - 1;
    return (size_t)items * Ww * TS * TS * (fp64 ? sizeof(double2) : sizeof(float2));
}

size_t degrid_scratch(const fr_plan *pl) { return scratch_round(planes_bytes(pl)); }

size_t grid_scratch(const fr_plan *pl) {
    int64_t items = 0;
    for (int64_t c = 0; c < pl->n_chan; ++c) items = std::max(items, pl->gwi_chan[c + 1] - pl->gwi_chan[c]);
    // values in record order (input-order calls; an upper bound for record-order ones)
    const size_t yrec = scratch_round((size_t)pl->n_vis * (pl->fp64 ? sizeof(double2) : sizeof(float2)));
    return scratch_round(planes_bytes(pl)) + scratch_round((size_t)vis_bound_blocks(pl->n_vis) * sizeof(float)) +
           yrec + scratch_round(grid_partial_bytes(items, pl->Ww, pl->W, pl->fp64));
}


// Device memory a plan build takes per visibility at its peak: the coordinate
// and key arrays of k_vis_coords (idx, cell, key, du, dv, dw, ph), the two key and
// permutation buffers of the sort and its tables (12 bytes per 16 keys), and the
// sorted records the plan keeps (idx, cell, du, dv, dw, ph, the record position
// of each visibility and the degridding pair lists), and the run flags of the
// sorted keys; per bucket, its first record and first gridding item, and the
// tile maps.
static size_t plan_bytes_per_vis(size_t rs) { return 12 + 4 * rs + 24 + 1 + 16 + 4 * rs + 1; }
static size_t plan_bytes_per_key() { return 8 + 4 + 4 + 1; }

// Bound on the device memory of building the coplanar doubled-field plan inside
// fr_make_psf_kernel: the records it keeps and its construction temporaries
// (per visibility: coordinates, keys, sort buffers), plus the per-bucket offsets.
size_t psf_plan_device_bound(const fr_plan *pl) {
    const size_t rs = pl->fp64 ? 8 : 4;
    const int64_t n_tiles = (4 * pl->nx / kTile) * (4 * pl->ny / kTile);
    const size_t n_keys = (size_t)pl->n_chan * n_tiles;
    return (size_t)pl->n_vis * (plan_bytes_per_vis(rs)) + (n_keys + 1) * plan_bytes_per_key();
}

// Bound on the arena scratch of gridding with the coplanar plan of the doubled
// field that fr_make_psf_kernel derives (built inside the call): one plane of
// 4 nx x 4 ny cells, the weighted values in record order, and the partial tiles
// of at most one gridding item per non-empty tile plus one per workgroup.
size_t psf_grid_scratch_bound(const fr_plan *pl) {
    const bool fp64 = pl->fp64;
    const int W = es_support(pl->eps, 2, 4);
    const int64_t nu = 4 * pl->nx, nv = 4 * pl->ny;
    const int64_t n_tiles = (nu / kTile) * (nv / kTile);
    // one item per non-empty bucket plus at most one more per workgroup
    const int64_t items = std::min<int64_t>(n_tiles, pl->n_row) +
                          std::min<int64_t>((int64_t)std::max(1, pl->ctx->n_cu) * grid_shape(W, 1, fp64).per_cu,
                                            std::max<int64_t>(1, (pl->n_row + kMinRangeRecords - 1) / kMinRangeRecords));
    const size_t planes = (size_t)nu * nv * (fp64 ? sizeof(double2) : sizeof(float2));
    return scratch_round(planes) + scratch_round((size_t)vis_bound_blocks(pl->n_vis) * sizeof(float)) +
           scratch_round((size_t)pl->n_vis * (fp64 ? sizeof(double2) : sizeof(float2))) +
           scratch_round(grid_partial_bytes(items, 1, W, fp64));
}

// forward: image channel -> planes (prep, row FFT, column FFT)
template <typename T>
// Only the tiles degridding reads are produced: the row pass stores the tile
// columns that hold an active tile, the column pass transforms those columns and
// stores the active tiles.
void image_to_planes(const fr_plan *pl, int64_t chan, const T *img_c, c2<T> *planes, hipStream_t st) {
    const int l2u = ilog2(pl->nu), l2v = ilog2(pl->nv);
    const int64_t c0 = pl->tcol_chan[chan], nc = pl->tcol_chan[chan + 1] - c0;
    if (nc == 0) return;  // no visibilities in this channel
    DegridRowPro<T> pro{img_c, pl->fac.as<T>(), pl->tpix.as<T>(), pl->tpix_w.as<double>(), pl->wplane.as<double>(),
                        (int)pl->nx, (int)pl->ny, (int)pl->nv, pl->coplanar ? 1 : 0, pl->taylor ? 1 : 0};
    DegridRowEpi<T> epi{planes, pl->col_active.as<uint8_t>() + chan * pl->ntv, (int)pl->nx, l2u, l2v};
    {
        ProfScope prof("wplane_rows_fwd", st);
        launch_fft_rows<T>(*pl->ctx, pro, epi, (int64_t)pl->n_planes * pl->nx, l2v, -1, st);
    }
    ProfScope prof("wplane_cols_fwd", st);
    launch_fft_cols<T>(*pl->ctx, BandColPro<T>{planes, (int)pl->nx, l2u, l2v},
                       ActiveColEpi<T>{planes, pl->tile_active.as<uint8_t>() + chan * pl->n_tiles, l2u, l2v, pl->ntv},
                       pl->n_planes, (int)pl->nv, l2u, (int)pl->nu, (int)pl->nu, -1, st, pl->tcol.as<int32_t>() + c0,
                       (int)nc, kTile);
}

// adjoint: planes -> image channel (inverse column FFT on the band, row kernel)
template <typename T>
// Only the tile columns that hold an active tile are transformed and read: the
// others are zero in every plane.
void planes_to_image(const fr_plan *pl, int64_t chan, const c2<T> *planes_c, T *img_c, hipStream_t st) {
    c2<T> *planes = const_cast<c2<T> *>(planes_c);
    const int l2u = ilog2(pl->nu), l2v = ilog2(pl->nv);
    const uint8_t *active = pl->tile_active.as<uint8_t>() + chan * pl->n_tiles;
    const uint8_t *col_active = pl->col_active.as<uint8_t>() + chan * pl->ntv;
    const int64_t c0 = pl->tcol_chan[chan], nc = pl->tcol_chan[chan + 1] - c0;
    {
        ProfScope prof("wplane_cols_inv", st);
        launch_fft_cols<T>(*pl->ctx, ActiveColPro<T>{planes, active, l2u, l2v, pl->ntv},
                           BandColEpi<T>{planes, (int)pl->nx, l2u, l2v},
                           pl->n_planes, (int)pl->nv, l2u, (int)pl->nu, (int)pl->nu, +1, st,
                           pl->tcol.as<int32_t>() + c0, (int)nc, kTile);
    }
    ProfScope prof("wplane_rows_inv", st);
    const int nv = (int)pl->nv;
    const size_t pl_line = (size_t)plen(nv) * sizeof(c2<T>), twb = (size_t)nv * sizeof(c2<T>);
    const int args_lines_small = std::max(1, std::min((int)pl->n_planes, 4096 / nv));
#define FR_GRID_ROWS(NT, TW, LINES)                                                                             \
    do {                                                                                                        \
        const size_t lds = (size_t)(LINES) * pl_line + ((TW) ? twb : 0);                                         \
        auto kern = k_grid_rows<T, NT, 4, 8, TW>;                                                               \
        allow_lds(kern, lds);                                                                                   \
        kern<<<dim3((unsigned)pl->nx), NT, lds, st>>>(planes, col_active, pl->n_planes, l2u, l2v, (int)pl->nx,   \
                                                      (int)pl->ny, pl->fac.as<T>(), pl->tpix.as<T>(),               \
                                                      pl->tpix_w.as<double>(),                                      \
                                                      pl->wplane.as<double>(),                                        \
                                                      pl->coplanar ? 1 : 0, pl->taylor ? 1 : 0, img_c, (LINES),       \
                                                      pl->ctx->tw<T>(l2v));                                           \
    } while (0)
    FR_REQUIRE(nv <= 64 * (nv <= 4096 ? 256 : 1024), "grid too large for the row pass");
    if (nv <= 4096) FR_GRID_ROWS(256, true, args_lines_small);
    else if (pl_line + twb <= (size_t)kLdsBytes) FR_GRID_ROWS(1024, true, 1);
    else FR_GRID_ROWS(1024, false, 1);
#undef FR_GRID_ROWS
    LAUNCH_CHECK();
}

template <typename T>
void degrid(const fr_plan *pl, const T *img, c2<T> *vis, hipStream_t st, const T *weight, bool sorted_out) {
    Scratch planes(planes_bytes(pl), st);
    const WorkItem *wis = pl->wi.as<WorkItem>();
    for (int64_t c = 0; c < pl->n_chan; ++c) {
        image_to_planes<T>(pl, c, img + c * pl->nx * pl->ny, planes.as<c2<T>>(), st);
        const int64_t w0 = pl->wi_chan[c], w1 = pl->wi_chan[c + 1];
        if (w1 > w0) {
#define FR_CALL_DEGRID(WW) \
    launch_degrid_w<T, WW>(pl, wis + w0, w1 - w0, planes.as<c2<T>>(), weight, vis, st, sorted_out ? 1 : 0)
            FR_W_DISPATCH(pl->W, FR_CALL_DEGRID)
#undef FR_CALL_DEGRID
        }
    }
}

template <typename T>
void grid(const fr_plan *pl, const c2<T> *vis, const T *weight, T *img, hipStream_t st, bool sorted_in) {
    Scratch planes(planes_bytes(pl), st);
    // bound on every gridded contribution (sets the fixed-point scale of the tiles);
    // values in input order are weighted and moved into record order on the way
    const int nbb = vis_bound_blocks(pl->n_vis);
    Scratch ybound((size_t)nbb * sizeof(float), st);
    Scratch yrec;
    const c2<T> *y_rec = vis;
    if (pl->n_vis > 0) {
        if (sorted_in) {
            k_vis_bound<T><<<dim3((unsigned)nbb), 256, 0, st>>>(vis, weight, pl->n_vis, ybound.as<float>());
        } else {
            yrec = Scratch((size_t)pl->n_vis * sizeof(c2<T>), st);
            y_rec = yrec.as<c2<T>>();
            k_vis_prepare<T><<<dim3((unsigned)nbb), 256, 0, st>>>(vis, weight, pl->r_pos.as<uint32_t>(), pl->n_vis,
                                                                  ybound.as<float>(), yrec.as<c2<T>>());
        }
        LAUNCH_CHECK();
    }
    for (int64_t c = 0; c < pl->n_chan; ++c) {
#define FR_CALL_GRID(WW) \
    launch_grid_w<T, WW>(pl, c, planes.as<c2<T>>(), y_rec, ybound.as<float>(), nbb, st, sorted_in ? 1 : 0)
        FR_W_DISPATCH(pl->W, FR_CALL_GRID)
#undef FR_CALL_GRID
        planes_to_image<T>(pl, c, planes.as<c2<T>>(), img + c * pl->nx * pl->ny, st);
    }
}

template void degrid<float>(const fr_plan *, const float *, float2 *, hipStream_t, const float *, bool);
template void degrid<double>(const fr_plan *, const double *, double2 *, hipStream_t, const double *, bool);
template void grid<float>(const fr_plan *, const float2 *, const float *, float *, hipStream_t, bool);
template void grid<double>(const fr_plan *, const double2 *, const double *, double *, hipStream_t, bool);

// ------------------------------------------------------------------ plan creation
static double n_minus_1(double l, double m) {
    const double r2 = l * l + m * m;
    return -r2 / (1.0 + std::sqrt(1.0 - r2));
}

// Chebyshev interpolant of a smooth function on [-h, h]
struct Cheb {
    std::vector<double> c;
    double h = 1;
    template <typename F> Cheb(F f, double h_, int n) : c(n), h(h_) {
        const double pi = 3.14159265358979323846;
        std::vector<double> fv(n);
        for (int k = 0; k < n; ++k) fv[k] = f(h * std::cos(pi * (k + 0.5) / n));
        for (int j = 0; j < n; ++j) {
            double s = 0;
            for (int k = 0; k < n; ++k) s += fv[k] * std::cos(pi * j * (k + 0.5) / n);
            c[j] = s * 2.0 / n;
        }
        c[0] *= 0.5;
    }
    double operator()(double x) const {
        const double t = x / h;
        double b1 = 0, b2 = 0;
        for (int j = (int)c.size() - 1; j >= 1; --j) {
            const double b0 = 2 * t * b1 - b2 + c[j];
            b2 = b1;
            b1 = b0;
        }
        return t * b1 - b2 + c[0];
    }
};

template <typename T> static DevBuf upload(const std::vector<double> &v) {
    std::vector<T> t(v.begin(), v.end());
    DevBuf b(t.size() * sizeof(T));
    HIP_CHECK(hipMemcpy(b.p, t.data(), b.bytes, hipMemcpyHostToDevice));
    return b;
}

// Gridding items and their workgroups.  A workgroup's time grows with its
// records, with the runs of equal base cell among them (each run ends in a flush
// of the register sums to the LDS tiles) and with its items (tile zeroing, band
// output, first loads); measured for the matrix-core spread at W = 7 with six
// planes on the VLA-like workload, a run costs about ten records and an item
// about 350.  The sorted records of each channel are cut into at most n_slots
// consecutive ranges (and at most one per kMinRangeRecords records, which keeps
// small channels to few items) of about equal cost, greedily with the smallest
// cap that needs no more ranges, so that one workgroup per slot finishes at
// about the same time; a range that crosses a bucket boundary takes one item per
// bucket piece.  Items stay in bucket order (gfirst[k]: first item of bucket k), and
// gseg holds per channel the first item of each range (from the channel's first
// item) followed by the channel's item count.
constexpr int64_t kCostRec = 10, kCostRun = 108, kCostItem = 4000;

static void grid_partition(const std::vector<int64_t> &bounds, const std::vector<uint8_t> &run_flag, int64_t n_chan,
                           int64_t keys_per_chan, int ntv, int n_tiles, int64_t n_slots, std::vector<WorkItem> &gwis,
                           std::vector<uint32_t> &gfirst, std::vector<int32_t> &gseg, std::vector<int64_t> &gwi_chan,
                           std::vector<int64_t> &gseg_chan) {
    const int64_t n_keys = n_chan * keys_per_chan;
    std::vector<int64_t> piece_key;
    gwi_chan.assign(n_chan + 1, 0);
    gseg_chan.assign(n_chan + 1, 0);
    for (int64_t c = 0; c < n_chan; ++c) {
        const int64_t k0 = c * keys_per_chan, k1 = k0 + keys_per_chan;
        const int64_t r0 = bounds[k0], r1 = bounds[k1];
        // runs started before each record of the channel
        std::vector<int64_t> R((size_t)(r1 - r0 + 1), 0);
        for (int64_t i = r0; i < r1; ++i) R[i - r0 + 1] = R[i - r0] + run_flag[i];
        auto cost = [&](int64_t a, int64_t b) { return kCostRec * (b - a) + kCostRun * (R[b - r0] - R[a - r0]); };
        std::vector<int64_t> nzb;
        int64_t total = 0;
        for (int64_t k = k0; k < k1; ++k)
            if (bounds[k + 1] > bounds[k]) {
                nzb.push_back(k);
                total += kCostItem + cost(bounds[k], bounds[k + 1]);
            }
        const int64_t item0 = (int64_t)gwis.size();
        // number of ranges for a cap of cap on each range's cost; emit: record them
        auto partition = [&](int64_t cap, bool emit) -> int64_t {
            int64_t n_rng = 0, used = 0;
            bool open = false;
            for (const int64_t k : nzb) {
                int64_t a = bounds[k];
                const int64_t b = bounds[k + 1];
                while (a < b) {
                    const int64_t room = cap - used - kCostItem;
                    int64_t e = a;
                    if (cost(a, b) <= room) {
                        e = b;
                    } else if (room >= 0) {
                        int64_t lo = a, hi = b;  // cost(a, lo) <= room < cost(a, hi)
                        while (hi - lo > 1) {
                            const int64_t mid = lo + (hi - lo) / 2;
                            if (cost(a, mid) <= room) lo = mid;
                            else hi = mid;
                        }
                        e = lo;
                    }
                    if (e == a) {
                        if (open) {  // full: the bucket continues in the next range
                            ++n_rng;
                            used = 0;
                            open = false;
                            continue;
                        }
                        e = a + 1;  // a range takes at least one record
                    }
                    if (emit) {
                        if (!open) gseg.push_back((int32_t)((int64_t)gwis.size() - item0));
                        const int64_t rem = k - k0;
                        const int p0 = (int)(rem / n_tiles), t = (int)(rem - (int64_t)p0 * n_tiles);
                        WorkItem w;
                        w.start = a;
                        w.count = (int32_t)(e - a);
                        w.tu = (t / ntv) * kTile;
                        w.tv = (t - (t / ntv) * ntv) * kTile;
                        w.p0 = p0;
                        w.chan = (int32_t)c;
                        w.rows = 0;
                        gwis.push_back(w);
                        piece_key.push_back(k);
                    }
                    used += kCostItem + cost(a, e);
                    open = true;
                    a = e;
                    if (a < b) {
                        ++n_rng;
                        used = 0;
                        open = false;
                    }
                }
            }
            return n_rng + (open ? 1 : 0);
        };
        if (!nzb.empty()) {
            // the smallest cap that needs at most n_rng ranges (a cap of total
            // needs one)
            const int64_t n_rng = std::max<int64_t>(
                1, std::min<int64_t>(n_slots, (r1 - r0 + kMinRangeRecords - 1) / kMinRangeRecords));
            int64_t lo = (total + n_rng - 1) / n_rng, hi = std::max(lo, total);
            while (lo < hi) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (partition(mid, false) <= n_rng) hi = mid;
                else lo = mid + 1;
            }
            partition(lo, true);
        }
        gseg.push_back((int32_t)((int64_t)gwis.size() - item0));
        gwi_chan[c + 1] = (int64_t)gwis.size();
        gseg_chan[c + 1] = (int64_t)gseg.size();
    }
    gfirst.assign(n_keys + 1, 0);
    int64_t it = 0;
    for (int64_t k = 0; k <= n_keys; ++k) {
        while (it < (int64_t)gwis.size() && piece_key[it] < k) ++it;
        gfirst[k] = (uint32_t)it;
    }
}

template <typename T>
static void build_records(fr_plan *pl, const DevBuf &d_uvw, const DevBuf &d_freq, int n_p0) {
    const int64_t n = pl->n_vis;
    const int ntu = (int)(pl->nu / kTile), ntv = (int)(pl->nv / kTile);
    const int n_tiles = ntu * ntv;
    pl->n_p0 = n_p0;
    pl->n_tiles = n_tiles;
    pl->ntu = ntu;
    pl->ntv = ntv;
    const int64_t n_keys = pl->n_chan * (int64_t)n_p0 * n_tiles;
    FR_REQUIRE(n_keys < (int64_t(1) << 32), "too many tiles x planes x channels");
    DevBuf key(n * 4), idx(n * 4), cell(n * 4), du(n * sizeof(T)), dv(n * sizeof(T)), dwf(n * sizeof(T)),
        ph(n * sizeof(T));
    const int64_t blocks = (n + 255) / 256;
    k_vis_coords<T><<<dim3((unsigned)blocks), 256>>>(
        d_uvw.as<double>(), d_freq.as<double>(), n, (int)pl->n_chan, ilog2(pl->nu), ilog2(pl->nv),
        pl->dx_, pl->dy_, pl->W, pl->Ww, pl->coplanar ? 1 : 0, pl->w0, pl->dw, pl->yc,
        2.0 * 3.14159265358979323846 * pl->taylor_h, pl->taylor ? 1 : 0, ntv, n_tiles, n_p0,
        key.as<uint32_t>(), idx.as<uint32_t>(), cell.as<uint32_t>(), du.as<T>(), dv.as<T>(), dwf.as<T>(), ph.as<T>());
    LAUNCH_CHECK();
    // stable radix sort of (bucket, cell in tile) keys (hand-written LSD sort, 8-bit
    // digits over the key's used bits); the permutation gathers the records
    DevBuf k64(n * 8), k64s(n * 8), perm(n * 4), perms(n * 4);
    k_sort_keys<<<dim3((unsigned)blocks), 256>>>(key.as<uint32_t>(), cell.as<uint32_t>(), n, k64.as<uint64_t>(),
                                                 perm.as<uint32_t>());
    LAUNCH_CHECK();
    int key_bits = 1;
    while ((int64_t(1) << key_bits) < n_keys) ++key_bits;
    const int end_bit = 10 + key_bits;
    DevBuf tmp(std::max<size_t>(RadixSortBuffers().bytes(n), 1));
    const bool in_second = radix_sort_pairs(k64.as<uint64_t>(), perm.as<uint32_t>(), k64s.as<uint64_t>(),
                                            perms.as<uint32_t>(), n, end_bit, tmp.p, nullptr);
    const uint64_t *keys_sorted = in_second ? k64s.as<uint64_t>() : k64.as<uint64_t>();
    const uint32_t *perm_sorted = in_second ? perms.as<uint32_t>() : perm.as<uint32_t>();
    DevBuf d_bounds((n_keys + 1) * 8);
    k_bucket_bounds<<<dim3((unsigned)((n_keys + 1 + 255) / 256)), 256>>>(keys_sorted, n, n_keys,
                                                                          d_bounds.as<int64_t>());
    LAUNCH_CHECK();
    std::vector<int64_t> bounds(n_keys + 1);
    HIP_CHECK(hipMemcpy(bounds.data(), d_bounds.p, d_bounds.bytes, hipMemcpyDeviceToHost));
    {
        DevBuf d_steps(sizeof(unsigned long long));
        HIP_CHECK(hipMemset(d_steps.p, 0, d_steps.bytes));
        k_count_runs<<<dim3((unsigned)((n + 255) / 256)), 256>>>(keys_sorted, n, d_steps.as<unsigned long long>());
        LAUNCH_CHECK();
        unsigned long long steps = 0;
        HIP_CHECK(hipMemcpy(&steps, d_steps.p, sizeof(steps), hipMemcpyDeviceToHost));
        pl->vis_per_run = (double)n / (double)(steps + 1);
    }
    // paired degridding: the sorted keys (bucket and base cell) on the host, to cut
    // the records into pairs of one base cell and the items at kPairsPerItem pairs
    const bool paired = paired_degrid(pl);
    pl->degrid_slots = paired ? 0 : n;
    std::vector<uint64_t> hkeys;
    std::vector<uint32_t> hpair;
    if (paired) {
        hkeys.resize(n);
        HIP_CHECK(hipMemcpy(hkeys.data(), keys_sorted, (size_t)n * 8, hipMemcpyDeviceToHost));
        hpair.assign(n, 0u);
    }
    int64_t run = 0;
    std::vector<WorkItem> wis;
    pl->wi_chan.assign(pl->n_chan + 1, 0);
    const int ch = chunk<T>();
    for (int64_t k = 0; k < n_keys; ++k) {
        const int64_t cnt = bounds[k + 1] - bounds[k];
        if (cnt) {
            const int64_t chan = k / ((int64_t)n_p0 * n_tiles);
            const int64_t rem = k - chan * n_p0 * n_tiles;
            const int p0 = (int)(rem / n_tiles);
            const int t = (int)(rem - (int64_t)p0 * n_tiles);
            const int tu = t / ntv, tv = t - tu * ntv;
            WorkItem w;
            w.tu = tu * kTile;
            w.tv = tv * kTile;
            w.p0 = p0;
            w.chan = (int32_t)chan;
            w.rows = 0;
            if (paired) {
                // consecutive records of one base cell two at a time (a record whose
                // successor has another cell, or lies beyond the item, alone); an item
                // ends after kPairsPerItem entries or ch records
                int64_t j = run;
                const int64_t end = run + cnt;
                while (j < end) {
                    w.start = j;
                    int entries = 0;
                    while (j < end && entries < kPairsPerItem && j - w.start < ch) {
                        const uint32_t a = (uint32_t)(j - w.start);
                        const bool two = j + 1 < end && j + 1 - w.start < ch && hkeys[j + 1] == hkeys[j];
                        hpair[w.start + entries] = a | ((two ? a + 1 : a) << 10) | (two ? 0u : (1u << 20));
                        ++entries;
                        j += two ? 2 : 1;
                    }
                    w.count = (int32_t)(j - w.start);
                    w.rows = entries;
                    pl->degrid_slots += entries;
                    wis.push_back(w);
                    pl->wi_chan[chan + 1] = (int64_t)wis.size();
                }
                w.rows = 0;
            } else {
                for (int64_t s = 0; s < cnt; s += ch) {
                    w.start = run + s;
                    w.count = (int32_t)std::min<int64_t>(ch, cnt - s);
                    wis.push_back(w);
                    pl->wi_chan[chan + 1] = (int64_t)wis.size();
                }
            }
        }
        run += cnt;
    }
    // gridding items and the workgroups that take them
    std::vector<WorkItem> gwis;
    std::vector<uint32_t> gfirst;
    std::vector<int32_t> gseg;
    {
        DevBuf d_flag((size_t)n);
        k_run_flags<<<dim3((unsigned)blocks), 256>>>(keys_sorted, 0, n, d_flag.as<uint8_t>());
        LAUNCH_CHECK();
        std::vector<uint8_t> flag((size_t)n);
        HIP_CHECK(hipMemcpy(flag.data(), d_flag.p, (size_t)n, hipMemcpyDeviceToHost));
        const GridShape gs = grid_shape(pl->W, pl->Ww, pl->fp64);
        const int64_t n_slots = (int64_t)std::max(1, pl->ctx->n_cu) * gs.per_cu;
        grid_partition(bounds, flag, pl->n_chan, (int64_t)n_p0 * n_tiles, ntv, n_tiles, n_slots, gwis, gfirst,
                       gseg, pl->gwi_chan, pl->gseg_chan);
    }
    {
        std::vector<uint8_t> act((size_t)pl->n_chan * n_tiles, 0);
        std::vector<int32_t> alist;
        pl->atile_chan.assign(pl->n_chan + 1, 0);
        for (int64_t c = 0; c < pl->n_chan; ++c) {
            uint8_t *a = act.data() + c * n_tiles;
            for (int p0 = 0; p0 < n_p0; ++p0)
                for (int t = 0; t < n_tiles; ++t) {
                    const int64_t k = (c * n_p0 + p0) * (int64_t)n_tiles + t;
                    if (gfirst[k + 1] == gfirst[k]) continue;
                    const int tu = t / ntv, tv = t - tu * ntv;
                    for (int di = 0; di < 2; ++di)
                        for (int dj = 0; dj < 2; ++dj) a[((tu + di) % ntu) * ntv + (tv + dj) % ntv] = 1;
                }
            for (int t = 0; t < n_tiles; ++t)
                if (a[t]) alist.push_back(t);
            pl->atile_chan[c + 1] = (int64_t)alist.size();
        }
        pl->atile = DevBuf(std::max<size_t>(1, alist.size()) * sizeof(int32_t));
        if (!alist.empty())
            HIP_CHECK(hipMemcpy(pl->atile.p, alist.data(), alist.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        pl->tile_active = DevBuf(act.size());
        HIP_CHECK(hipMemcpy(pl->tile_active.p, act.data(), act.size(), hipMemcpyHostToDevice));
        std::vector<uint8_t> cact((size_t)pl->n_chan * ntv, 0);
        std::vector<int32_t> clist;
        pl->tcol_chan.assign(pl->n_chan + 1, 0);
        for (int64_t c = 0; c < pl->n_chan; ++c) {
            for (int t = 0; t < n_tiles; ++t)
                if (act[c * n_tiles + t]) cact[c * ntv + t % ntv] = 1;
            for (int tv = 0; tv < ntv; ++tv)
                if (cact[c * ntv + tv]) clist.push_back(tv);
            pl->tcol_chan[c + 1] = (int64_t)clist.size();
        }
        pl->col_active = DevBuf(cact.size());
        HIP_CHECK(hipMemcpy(pl->col_active.p, cact.data(), cact.size(), hipMemcpyHostToDevice));
        pl->tcol = DevBuf(std::max<size_t>(1, clist.size()) * sizeof(int32_t));
        if (!clist.empty())
            HIP_CHECK(hipMemcpy(pl->tcol.p, clist.data(), clist.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    for (int64_t c = 1; c <= pl->n_chan; ++c) pl->wi_chan[c] = std::max(pl->wi_chan[c], pl->wi_chan[c - 1]);
    pl->n_gwi = (int64_t)gwis.size();
    pl->gseg = DevBuf(gseg.size() * sizeof(int32_t));
    HIP_CHECK(hipMemcpy(pl->gseg.p, gseg.data(), pl->gseg.bytes, hipMemcpyHostToDevice));
    pl->gwi = DevBuf(std::max<size_t>(1, gwis.size()) * sizeof(WorkItem));
    if (!gwis.empty())
        HIP_CHECK(hipMemcpy(pl->gwi.p, gwis.data(), gwis.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    pl->gkey_first = DevBuf(gfirst.size() * sizeof(uint32_t));
    HIP_CHECK(hipMemcpy(pl->gkey_first.p, gfirst.data(), pl->gkey_first.bytes, hipMemcpyHostToDevice));
    pl->r_idx = DevBuf(n * 4);
    pl->r_cell = DevBuf(n * 4);
    pl->r_du = DevBuf(n * sizeof(T));
    pl->r_dv = DevBuf(n * sizeof(T));
    pl->r_dw = DevBuf(n * sizeof(T));
    pl->r_ph = DevBuf(n * sizeof(T));
    pl->r_pos = DevBuf(n * 4);
    k_gather_records<T><<<dim3((unsigned)blocks), 256>>>(
        n, perm_sorted, idx.as<uint32_t>(), cell.as<uint32_t>(), du.as<T>(), dv.as<T>(), dwf.as<T>(),
        ph.as<T>(), pl->r_idx.as<uint32_t>(), pl->r_cell.as<uint32_t>(), pl->r_du.as<T>(), pl->r_dv.as<T>(),
        pl->r_dw.as<T>(), pl->r_ph.as<T>(), pl->r_pos.as<uint32_t>());
    LAUNCH_CHECK();
    if (pl->n_gwi > 0) {
        k_item_rows<<<dim3((unsigned)((pl->n_gwi + 255) / 256)), 256>>>(pl->gwi.as<WorkItem>(), pl->n_gwi,
                                                                         pl->r_cell.as<uint32_t>(), pl->W);
        LAUNCH_CHECK();
    }
    pl->n_wi = (int64_t)wis.size();
    pl->wi = DevBuf(std::max<size_t>(1, wis.size()) * sizeof(WorkItem));
    if (!wis.empty()) HIP_CHECK(hipMemcpy(pl->wi.p, wis.data(), wis.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    if (paired) {
        pl->dpair = DevBuf((size_t)n * 4);
        HIP_CHECK(hipMemcpy(pl->dpair.p, hpair.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    }
    HIP_CHECK(hipDeviceSynchronize());
}

// ------------------------------------------------------------------ inspection
int64_t plan_n_keys(const fr_plan *pl) { return pl->n_chan * (int64_t)pl->n_p0 * pl->n_tiles; }

template <typename T> static void export_keys(const fr_plan *pl, uint64_t *keys_host) {
    const int64_t n = pl->n_vis;
    DevBuf d_uvw(pl->n_row * 3 * sizeof(double)), d_freq(pl->n_chan * sizeof(double));
    HIP_CHECK(hipMemcpy(d_uvw.p, pl->uvw_host.data(), d_uvw.bytes, hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(d_freq.p, pl->freq.data(), d_freq.bytes, hipMemcpyHostToDevice));
    DevBuf key(n * 4), idx(n * 4), cell(n * 4), du(n * sizeof(T)), dv(n * sizeof(T)), dwf(n * sizeof(T)),
        ph(n * sizeof(T)), k64(n * 8), perm(n * 4);
    const int64_t blocks = (n + 255) / 256;
    k_vis_coords<T><<<dim3((unsigned)blocks), 256>>>(
        d_uvw.as<double>(), d_freq.as<double>(), n, (int)pl->n_chan, ilog2(pl->nu), ilog2(pl->nv), pl->dx_, pl->dy_,
        pl->W, pl->Ww, pl->coplanar ? 1 : 0, pl->w0, pl->dw, pl->yc, 2.0 * 3.14159265358979323846 * pl->taylor_h,
        pl->taylor ? 1 : 0, pl->ntv, pl->n_tiles, pl->n_p0, key.as<uint32_t>(), idx.as<uint32_t>(),
        cell.as<uint32_t>(), du.as<T>(), dv.as<T>(), dwf.as<T>(), ph.as<T>());
    LAUNCH_CHECK();
    k_sort_keys<<<dim3((unsigned)blocks), 256>>>(key.as<uint32_t>(), cell.as<uint32_t>(), n, k64.as<uint64_t>(),
                                                 perm.as<uint32_t>());
    LAUNCH_CHECK();
    HIP_CHECK(hipMemcpy(keys_host, k64.p, n * 8, hipMemcpyDeviceToHost));
}

// Bucket boundaries from a list of work items (chunks of one bucket each, in bucket
// order), checking that the items of every bucket tile its range exactly.
static void bounds_from_items(const fr_plan *pl, const DevBuf &items, int64_t n_items, int64_t *bs) {
    const int64_t n_keys = plan_n_keys(pl);
    std::vector<WorkItem> it(n_items);
    if (n_items) HIP_CHECK(hipMemcpy(it.data(), items.p, n_items * sizeof(WorkItem), hipMemcpyDeviceToHost));
    int64_t end = 0, k_next = 0;
    for (int64_t j = 0; j < n_items; ++j) {
        const WorkItem &w = it[j];
        const int64_t k = ((int64_t)w.chan * pl->n_p0 + w.p0) * pl->n_tiles + (int64_t)(w.tu / kTile) * pl->ntv +
                          w.tv / kTile;
        if (k >= k_next) {  // first item of bucket k: the buckets in between are empty
            if (w.start != end) throw Error(FR_EHIP, "work items leave a gap in the sorted records");
            for (; k_next <= k; ++k_next) bs[k_next] = end;
        } else if (k != k_next - 1 || w.start != end) {
            throw Error(FR_EHIP, "work items out of bucket order");
        }
        end = w.start + w.count;
    }
    if (end != pl->n_vis) throw Error(FR_EHIP, "work items do not cover every record");
    for (; k_next <= n_keys; ++k_next) bs[k_next] = end;
}

void plan_export_order(const fr_plan *pl, uint64_t *keys, uint32_t *perm, int64_t *bucket_start) {
    const int64_t n = pl->n_vis;
    if (keys && n) {
        if (pl->fp64) export_keys<double>(pl, keys);
        else export_keys<float>(pl, keys);
    }
    if (perm && n) {
        HIP_CHECK(hipMemcpy(perm, pl->r_idx.p, n * 4, hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < n; ++k) perm[k] &= 0x7fffffffu;
    }
    if (bucket_start) {
        bounds_from_items(pl, pl->wi, pl->n_wi, bucket_start);
        std::vector<int64_t> g(plan_n_keys(pl) + 1);
        bounds_from_items(pl, pl->gwi, pl->n_gwi, g.data());
        for (size_t k = 0; k < g.size(); ++k)
            if (g[k] != bucket_start[k]) throw Error(FR_EHIP, "degridding and gridding items disagree");
    }
}

void plan_build(fr_plan *pl, const double *uvw_m, const double *freq_hz) {
    const int64_t nx = pl->nx, ny = pl->ny;
    // --- kernel support and shape
    // w extent after folding every visibility to w >= 0
    double wmin = 0, wmax = 0;
    {
        double amin = INFINITY, amax = 0;
        for (int64_t r = 0; r < pl->n_row; ++r) {
            const double a = std::fabs(uvw_m[3 * r + 2]);
            amin = std::min(amin, a);
            amax = std::max(amax, a);
        }
        double fmin = INFINITY, fmax = 0;
        for (double f : pl->freq) {
            fmin = std::min(fmin, f);
            fmax = std::max(fmax, f);
        }
        if (pl->n_row == 0) amin = amax = 0;
        wmin = amin * fmin / kCLight;
        wmax = amax * fmax / kCLight;
    }
    const double lmax = (nx / 2) * pl->dx_, mmax = (ny / 2) * pl->dy_;
    const double ymin = n_minus_1(lmax, mmax);  // most negative n - 1 over the image
    const bool coplanar = pl->coplanar || wmax * std::fabs(ymin) == 0.0;
    pl->coplanar = coplanar;
    const int dims = coplanar ? 2 : 3;
    pl->W = es_support(pl->eps, dims, 4);
    pl->beta = es_beta(pl->W);
    pl->eps_bound = dims * kESAliasBound[pl->W];
    ESKernel kuv(pl->W, pl->beta);
    if (coplanar) {
        pl->Ww = 1;
        pl->wbeta = 0;
        pl->n_planes = 1;
        pl->w0 = 0;
        pl->dw = 1;
        pl->yc = 0;
    } else {
        const double h = -ymin / 2;  // (n - 1) - yc lies in [-h, h]
        pl->yc = ymin / 2;
        // With w0 = wmin - (Ww/2 - 1 + delta) dw, the first plane a visibility
        // touches is ceil((w - wmin)/dw + delta - 1), so delta in (0, 1] can be
        // chosen to centre the w-range inside the fewest first-plane slots:
        // n_p0 = max(1, ceil(range/dw)) planes of origin, Ww - 1 more planes.
        auto layout = [&](double dw_, double &delta, int &n_p0) {
            const double f = (wmax - wmin) / dw_;
            const double cf = std::ceil(f);
            if (cf - f > 1e-6) {
                delta = 0.5 * (cf - f);
                n_p0 = std::max(1, (int)cf);
            } else {
                delta = 1.0;  // range is a whole number of planes (or zero)
                n_p0 = (int)cf + 1;
            }
        };
        // The kernel along w: support Ww, shape and plane spacing dw = xmax / h
        // chosen together for the fewest planes n_p0 + Ww - 1 whose aliasing bound
        // fits the accuracy the uv kernel leaves (then the narrower kernel, then the
        // coarser grid); the 2x-oversampled kernel of the uv support always fits.
        const double eps_w = pl->eps - 2 * kESAliasBound[pl->W];
        int best_npl = INT32_MAX, best_ww = pl->W, best_x = 0;
        for (int ww = 4; ww <= pl->W; ++ww)
            for (int xi = 0; xi < 5; ++xi) {
                if (kESwTable[ww][xi].bound > eps_w && !(ww == pl->W && xi == 0)) continue;
                double dl = 1.0;
                int p0 = 1;
                layout(kESwXmax[xi] / h, dl, p0);
                const int npl_c = p0 + ww - 1;
                if (npl_c < best_npl || (npl_c == best_npl && ww < best_ww)) {
                    best_npl = npl_c;
                    best_ww = ww;
                    best_x = xi;
                }
            }
        pl->Ww = best_ww;
        pl->wbeta = best_ww == pl->W && best_x == 0 ? pl->beta : kESwTable[best_ww][best_x].beta_over_w * best_ww;
        pl->w_xmax = kESwXmax[best_x];
        pl->eps_bound = 2 * kESAliasBound[pl->W] +
                        (best_ww == pl->W && best_x == 0 ? kESAliasBound[pl->W] : kESwTable[best_ww][best_x].bound);
        double dw = pl->w_xmax / h;
        double delta = 1.0;
        int n_p0 = 1;
        layout(dw, delta, n_p0);
        int npl = n_p0 + pl->Ww - 1;
        if (pl->n_wplanes_req > 0) {
            FR_REQUIRE(pl->n_wplanes_req >= npl, "n_wplanes is below the minimum for this epsilon (" +
                                                     std::to_string(npl) + ")");
            // spend the extra planes on a finer w-grid (larger oversampling in w)
            const int want_p0 = pl->n_wplanes_req - pl->Ww + 1;
            if (wmax > wmin && want_p0 > 1) dw = std::min(dw, (wmax - wmin) / (want_p0 - 0.5));
            layout(dw, delta, n_p0);
            npl = pl->n_wplanes_req;
        }
        pl->dw = dw;
        pl->n_planes = npl;
        pl->w0 = wmin - (0.5 * pl->Ww - 1.0 + delta) * dw;
        // Taylor expansion in w: exp(-2 pi i w t) = sum_j x^j / j! (-i t / h)^j with
        // x = 2 pi w h <= x_max; J + 1 terms leave x_max^(J+1) / (J+1)! of it, kept
        // below epsilon / 8 (the uv kernel keeps 2 dimensions of the rest).  Only
        // for x_max <= 1, where no term exceeds 1 (no cancellation between terms).
        const double x_max = 2.0 * 3.14159265358979323846 * wmax * h;
        if (pl->want_taylor && pl->n_wplanes_req == 0 && x_max <= 1.0) {
            int J = 0;
            double rem = x_max;  // x_max^(J+1) / (J+1)!
            while (rem > pl->eps / 8 && J < 15) {
                ++J;
                rem *= x_max / (J + 1);
            }
            if (J + 1 < npl) {
                pl->taylor = true;
                pl->taylor_h = h;
                pl->W = es_support(pl->eps * 7.0 / 8.0, 2, 4);
                pl->beta = es_beta(pl->W);
                pl->eps_bound = 2 * kESAliasBound[pl->W] + rem;
                kuv = ESKernel(pl->W, pl->beta);
                pl->Ww = J + 1;
                pl->wbeta = 0;
                pl->n_planes = J + 1;
                pl->w0 = 0;
                pl->dw = 1;
            }
        }
    }
    ESKernel kw(pl->Ww > 1 && !pl->taylor ? pl->Ww : 4, pl->Ww > 1 && !pl->taylor ? pl->wbeta : 9.2);
    // the w correction is evaluated at xi = dw t, |xi| <= h dw (<= w_xmax, less when
    // extra planes refined the grid)
    // --- per-pixel factors
    std::vector<double> cu(nx), cv(ny);
    for (int64_t i = 0; i < nx; ++i) cu[i] = 1.0 / kuv.psi_hat((double)(i - nx / 2) / (double)pl->nu);
    for (int64_t j = 0; j < ny; ++j) cv[j] = 1.0 / kuv.psi_hat((double)(j - ny / 2) / (double)pl->nv);
    std::vector<double> fac(nx * ny), tpix(nx * ny, 0.0), tpix_w(nx * ny, 0.0), nfac(nx * ny);
    Cheb psiw([&](double t) { return kw.psi_hat(t); }, pl->w_xmax, 40);
    for (int64_t i = 0; i < nx; ++i) {
        const double l = (double)(i - nx / 2) * pl->dx_;
        for (int64_t j = 0; j < ny; ++j) {
            const double m = (double)(j - ny / 2) * pl->dy_;
            const double y = n_minus_1(l, m);
            const double a = pl->divide_by_n ? 1.0 / (1.0 + y) : 1.0;
            double f = a * cu[i] * cv[j];
            if (pl->taylor) {
                tpix[i * ny + j] = (y - pl->yc) / pl->taylor_h;
            } else if (!coplanar) {
                const double t = y - pl->yc;
                tpix_w[i * ny + j] = t;
                f /= psiw(pl->dw * t);
            }
            fac[i * ny + j] = f;
            nfac[i * ny + j] = a;
        }
    }
    std::vector<double> wpl(pl->n_planes);
    for (int p = 0; p < pl->n_planes; ++p) wpl[p] = coplanar || pl->taylor ? 0.0 : pl->w0 + p * pl->dw;
    if (pl->fp64) {
        pl->fac = upload<double>(fac);
        if (pl->taylor) pl->tpix = upload<double>(tpix);
        pl->nfac = upload<double>(nfac);
    } else {
        pl->fac = upload<float>(fac);
        if (pl->taylor) pl->tpix = upload<float>(tpix);
        pl->nfac = upload<float>(nfac);
    }
    // w-stacked plans of either precision keep (n - 1) - yc in double: the plane
    // phases w_p t are formed and reduced modulo one cycle in double
    if (!coplanar && !pl->taylor) pl->tpix_w = upload<double>(tpix_w);
    pl->wplane = upload<double>(wpl);
    // --- visibility records
    DevBuf d_uvw(std::max<int64_t>(1, pl->n_row) * 3 * sizeof(double));
    DevBuf d_freq(pl->n_chan * sizeof(double));
    if (pl->n_row) HIP_CHECK(hipMemcpy(d_uvw.p, uvw_m, pl->n_row * 3 * sizeof(double), hipMemcpyHostToDevice));
    HIP_CHECK(hipMemcpy(d_freq.p, pl->freq.data(), d_freq.bytes, hipMemcpyHostToDevice));
    const int n_p0 = pl->n_planes - pl->Ww + 1;
    if (pl->n_vis > 0) {
        if (pl->fp64) build_records<double>(pl, d_uvw, d_freq, n_p0);
        else build_records<float>(pl, d_uvw, d_freq, n_p0);
    } else {
        pl->wi_chan.assign(pl->n_chan + 1, 0);
        pl->gwi_chan.assign(pl->n_chan + 1, 0);
        pl->gseg_chan.assign(pl->n_chan + 1, 0);
        pl->n_p0 = n_p0;
        pl->ntu = (int)(pl->nu / kTile);
        pl->ntv = (int)(pl->nv / kTile);
        pl->n_tiles = pl->ntu * pl->ntv;
        // no active tile anywhere: gridding yields zero images without reading the planes
        pl->atile_chan.assign(pl->n_chan + 1, 0);
        pl->atile = DevBuf(sizeof(int32_t));
        pl->tile_active = DevBuf((size_t)pl->n_chan * pl->n_tiles);
        HIP_CHECK(hipMemset(pl->tile_active.p, 0, pl->tile_active.bytes));
        pl->col_active = DevBuf((size_t)pl->n_chan * pl->ntv);
        HIP_CHECK(hipMemset(pl->col_active.p, 0, pl->col_active.bytes));
        pl->tcol = DevBuf(sizeof(int32_t));
        pl->tcol_chan.assign(pl->n_chan + 1, 0);
    }
    pl->resident = pl->fac.bytes + pl->tpix.bytes + pl->tpix_w.bytes + pl->nfac.bytes + pl->wplane.bytes + pl->r_idx.bytes +
                   pl->r_cell.bytes + pl->r_du.bytes + pl->r_dv.bytes + pl->r_dw.bytes + pl->r_ph.bytes + pl->r_pos.bytes +
                   pl->dpair.bytes +
                   pl->wi.bytes + pl->gwi.bytes + pl->gseg.bytes + pl->gkey_first.bytes + pl->atile.bytes +
                   pl->tile_active.bytes + pl->col_active.bytes + pl->tcol.bytes;
}

}  // namespace frmi
