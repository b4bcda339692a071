// FFT convolutions with real, even kernels on real images (PSF convolution of
// Sec. 3.3.2 on the zero-padded doubled grid, periodic noise and prior
// convolutions of Sec. 3.3.3), as three LDS-resident passes:
//
//   1. rows:    real rows of length 2M (only the first n_in values non-zero) ->
//               packed half-spectrum rows of M complex values (half-length trick;
//               the real DC and Nyquist values share slot 0);
//   2. columns: strips of C packed columns; forward FFT of length Lc (input rows
//               beyond n_in are zero), multiply (or divide) by the kernel column,
//               inverse FFT, keep the first n_out rows;
//   3. rows:    inverse of pass 1, keep the first n_out_cols real outputs.
//
// The kernel K is real with Hermitian symmetry K[-k] = K[k]; slot 0 of a packed
// row carries two independent real columns (DC and Nyquist), which the column
// pass separates with the usual even/odd split before multiplying each by its
// own kernel column.  Overall scaling 1/(Lc M) makes the pipeline equal to
// irfft2(K rfft2(x)) with numpy's normalisation.
//
// Prologue/epilogue functors let callers fuse elementwise work (1/n factors,
// exp(s), residuals, gradient products) into the first and last pass.
#pragma once

#include <type_traits>

#include "fft.h"

namespace frmi {

// A row prologue may carry per-block set-up: `bool begin()` runs once per
// workgroup before any element is loaded (every thread calls it; it may use
// barriers) and returns false to skip the block's work.
template <class P, class = void> struct has_begin : std::false_type {};
template <class P> struct has_begin<P, std::void_t<decltype(std::declval<P &>().begin())>> : std::true_type {};

// ------------------------------------------------------------------ pass 1
template <typename T, int NTHR, int BPT, bool TWL, class Pro, int ODD = 1>
__global__ __launch_bounds__(NTHR) void k_rfft_rows(Pro pro_arg, c2<T> *__restrict__ Y, int64_t nrows,
                                                     int log2M, int n_in, int lines_per_wg,
                                                     const c2<T> *__restrict__ tw,
                                                     const c2<T> *__restrict__ tw2) {
    Pro pro = pro_arg;
    if constexpr (has_begin<Pro>::value) {
        if (!pro.begin()) return;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int M = ODD << log2M;
    const int64_t row0 = (int64_t)blockIdx.x * lines_per_wg;
    const int nl = (int)min<int64_t>(lines_per_wg, nrows - row0);
    const int ld = plen(M);
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + lines_per_wg * ld, tw, M);
    staged_copy<NTHR>(
        nl * M,
        [&](int idx) {
            const int c = line_of<ODD>(idx, log2M), e = elem_of<ODD>(idx, c, M);
            c2<T> z = mk<T>(T(0), T(0));
            if (2 * e < n_in) {
                z.x = pro(row0 + c, 2 * e);
                z.y = pro(row0 + c, 2 * e + 1);
            }
            return z;
        },
        [&](int idx, c2<T> v) {
            const int c = line_of<ODD>(idx, log2M);
            buf[c * ld + padx(elem_of<ODD>(idx, c, M))] = v;
        });
    __syncthreads();
    lds_fft<T, NTHR, BPT, ODD>(buf, ld, nl, log2M, -1, twp);
    const int half = M / 2 + 1;
    for (int c = 0; c < nl; ++c)
    for (int k = threadIdx.x; k < half; k += NTHR) {
        c2<T> *line = buf + c * ld;
        if (k == 0) {
            c2<T> z = line[0];
            line[0] = mk<T>(z.x + z.y, z.x - z.y);
        } else {
            const int km = M - k;
            c2<T> a = line[padx(k)], b = line[padx(km)];
            c2<T> E = mk<T>((a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5));
            c2<T> O = mk<T>((a.y + b.y) * T(0.5), (b.x - a.x) * T(0.5));
            line[padx(k)] = cadd<T>(E, cmul<T>(tw2[k], O));
            if (km != k) line[padx(km)] = cadd<T>(cconj<T>(E), cmul<T>(tw2[km], cconj<T>(O)));
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nl * M; idx += NTHR) {
        const int c = line_of<ODD>(idx, log2M);
        Y[row0 * M + idx] = buf[c * ld + padx(elem_of<ODD>(idx, c, M))];
    }
}

// ------------------------------------------------------------------ pass 2
// Factor applied per frequency: mode 0: K, 1: 1/K, 2: sqrt K, 3: 1/sqrt K.
template <typename T> __device__ __forceinline__ T kernel_factor(T k, int mode) {
    if (mode == 0) return k;
    if (mode == 1) return T(1) / k;
    const T r = sqrt(k);
    return mode == 2 ? r : T(1) / r;
}

// K: [nk][Lc][M + 1] real, image g uses kernel g % nk, or K_alt [Lc][M + 1] for
// images g >= g_alt; `mode` as kernel_factor.  M: packed row width; Lc = ODD
// 2^log2Lc.  A non-zero *skip (device flag, optional) turns the launch into a no-op.
template <typename T, int NTHR, int BPT, bool TWL, int ODD = 1>
__global__ __launch_bounds__(NTHR) void k_conv_cols(c2<T> *__restrict__ Y, int M, int log2Lc,
                                                     int n_in, int n_out, int C,
                                                     const T *__restrict__ K, int nk, int mode,
                                                     T scale, const c2<T> *__restrict__ tw,
                                                     const T *__restrict__ K_alt, int64_t g_alt,
                                                     const int *__restrict__ skip) {
    if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int Lc = ODD << log2Lc;
    const int ld = plen(Lc) + 1;
    const unsigned w = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int col0 = (int)(w % gridDim.x) * C;
    const int64_t g = w / gridDim.x;
    const int log2C = 31 - __builtin_clz(C);  // strips are a power of two wide
    c2<T> *Yg = Y + g * n_in * (int64_t)M;  // packed rows of image g (n_in rows stored)
    const T *Kg = g >= g_alt ? K_alt : K + (g % nk) * (int64_t)Lc * (M + 1);
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + C * ld, tw, Lc);
    staged_copy<NTHR>(
        C * Lc,
        [&](int idx) {
            const int r = idx >> log2C, c = idx & (C - 1);
            return (r < n_in) ? Yg[(int64_t)r * M + col0 + c] : mk<T>(T(0), T(0));
        },
        [&](int idx, c2<T> v) {
            const int r = idx >> log2C, c = idx & (C - 1);
            buf[c * ld + padx(r)] = v;
        });
    __syncthreads();
    lds_fft<T, NTHR, BPT, ODD>(buf, ld, C, log2Lc, -1, twp);
    // column fastest: the C kernel values of a row k are adjacent in memory, so a
    // strip reads K in row segments rather than one scattered element per thread
    for (int idx = threadIdx.x; idx < C * Lc; idx += NTHR) {
        const int k = idx >> log2C, c = idx & (C - 1);
        const int col = col0 + c;
        if (col == 0) {
            // slot 0 = DC column + i * Nyquist column: split, scale each, recombine
            if (k <= Lc / 2) {
                const int km = k ? Lc - k : 0;
                c2<T> a = buf[padx(k)], b = buf[padx(km)];
                // A = (F[k] + conj F[-k]) / 2,  Bn = (F[k] - conj F[-k]) / 2i
                c2<T> A = mk<T>((a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5));
                c2<T> Bn = mk<T>((a.y + b.y) * T(0.5), (b.x - a.x) * T(0.5));
                T k0 = Kg[(int64_t)k * (M + 1)], k1 = Kg[(int64_t)k * (M + 1) + M];
                T k0m = Kg[(int64_t)km * (M + 1)], k1m = Kg[(int64_t)km * (M + 1) + M];
                k0 = kernel_factor(k0, mode) * scale;
                k1 = kernel_factor(k1, mode) * scale;
                k0m = kernel_factor(k0m, mode) * scale;
                k1m = kernel_factor(k1m, mode) * scale;
                // F'[k] = A k0 + i Bn k1 ; F'[-k] = conj(A) k0m + i conj(Bn) k1m
                buf[padx(k)] = mk<T>(A.x * k0 - Bn.y * k1, A.y * k0 + Bn.x * k1);
                if (km != k) buf[padx(km)] = mk<T>(A.x * k0m + Bn.y * k1m, -A.y * k0m + Bn.x * k1m);
            }
        } else {
            T kv = Kg[(int64_t)k * (M + 1) + col];
            kv = kernel_factor(kv, mode) * scale;
            c2<T> v = buf[c * ld + padx(k)];
            buf[c * ld + padx(k)] = mk<T>(v.x * kv, v.y * kv);
        }
    }
    __syncthreads();
    lds_fft<T, NTHR, BPT, ODD>(buf, ld, C, log2Lc, +1, twp);
    for (int idx = threadIdx.x; idx < C * n_out; idx += NTHR) {
        const int r = idx >> log2C, c = idx & (C - 1);
        Yg[(int64_t)r * M + col0 + c] = buf[c * ld + padx(r)];
    }
}

// ------------------------------------------------------------------ pass 3
// Packed half-spectrum lines (M complex values each; slot 0 holds the real DC and
// Nyquist values) -> the spectra of the complex lines z[e] = x[2e] + i x[2e + 1]
// whose inverse FFT gives the real rows (inverse of the half-length trick).
template <typename T, int NTHR>
__device__ __forceinline__ void irfft_unpack(c2<T> *buf, int ld, int nl, int M, const c2<T> *__restrict__ tw2) {
    const int half = M / 2 + 1;
    for (int c = 0; c < nl; ++c)
    for (int k = threadIdx.x; k < half; k += NTHR) {
        c2<T> *line = buf + c * ld;
        if (k == 0) {
            c2<T> p = line[0];
            line[0] = mk<T>((p.x + p.y) * T(0.5), (p.x - p.y) * T(0.5));
        } else {
            const int km = M - k;
            c2<T> a = line[padx(k)], b = line[padx(km)];
            c2<T> E = mk<T>((a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5));
            c2<T> D = mk<T>((a.x - b.x) * T(0.5), (a.y + b.y) * T(0.5));
            c2<T> O = cmul<T>(D, cconj<T>(tw2[k]));
            line[padx(k)] = mk<T>(E.x - O.y, E.y + O.x);
            if (km != k) {
                c2<T> Ep = cconj<T>(E);
                c2<T> Op = cmul<T>(mk<T>(-D.x, D.y), cconj<T>(tw2[km]));
                line[padx(km)] = mk<T>(Ep.x - Op.y, Ep.y + Op.x);
            }
        }
    }
}

template <typename T, int NTHR, int BPT, bool TWL, class Epi, int ODD = 1>
__global__ __launch_bounds__(NTHR) void k_irfft_rows(Epi epi, const c2<T> *__restrict__ Y, int64_t nrows,
                                                      int log2M, int n_out_cols, int lines_per_wg,
                                                      const c2<T> *__restrict__ tw,
                                                      const c2<T> *__restrict__ tw2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int M = ODD << log2M;
    const int64_t row0 = (int64_t)blockIdx.x * lines_per_wg;
    const int nl = (int)min<int64_t>(lines_per_wg, nrows - row0);
    const int ld = plen(M);
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + lines_per_wg * ld, tw, M);
    staged_copy<NTHR>(
        nl * M, [&](int idx) { return Y[row0 * M + idx]; },
        [&](int idx, c2<T> v) {
            const int c = line_of<ODD>(idx, log2M);
            buf[c * ld + padx(elem_of<ODD>(idx, c, M))] = v;
        });
    __syncthreads();
    irfft_unpack<T, NTHR>(buf, ld, nl, M, tw2);
    __syncthreads();
    lds_fft<T, NTHR, BPT, ODD>(buf, ld, nl, log2M, +1, twp);
    const int npair = n_out_cols / 2;
    for (int c = 0; c < nl; ++c)
        for (int e = threadIdx.x; e < npair; e += NTHR) {
            c2<T> z = buf[c * ld + padx(e)];
            epi(row0 + c, 2 * e, z.x, z.y);
        }
}


// Sum of v over the workgroup (NTHR threads), FP64, fixed order; valid in thread 0.
template <int NTHR> __device__ __forceinline__ double block_sum_n(double v) {
    __shared__ double sh[NTHR / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NTHR / 64; ++k) t += sh[k];
    return t;
}

// Pass 3 over pairs of images: row r of the first n_rows packed rows goes with
// row r + pair_offset (NPART = 2; NPART = 1 has no partner), both inverse
// transformed in the same workgroup so that the epilogue sees the two real
// values of a pixel together: epi(r, col, a0, a1, b0, b1) receives columns col
// and col + 1 of the row and of its partner, stores what it needs and returns a
// contribution to a sum; partials[blockIdx.x] gets the workgroup's FP64 sum.
// A non-zero *skip turns the launch into a no-op.
template <typename T, int NTHR, int BPT, bool TWL, class Epi, int NPART>
__global__ __launch_bounds__(NTHR) void k_irfft_rows_pair(Epi epi, const c2<T> *__restrict__ Y, int64_t n_rows,
                                                           int64_t pair_offset, int log2M, int n_out_cols,
                                                           int lines_per_wg, const c2<T> *__restrict__ tw,
                                                           const c2<T> *__restrict__ tw2,
                                                           double *__restrict__ partials,
                                                           const int *__restrict__ skip) {
    if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int M = 1 << log2M;
    const int64_t row0 = (int64_t)blockIdx.x * lines_per_wg;
    const int nl = (int)min<int64_t>(lines_per_wg, n_rows - row0);
    const int ld = plen(M);
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + NPART * lines_per_wg * ld, tw, M);
    staged_copy<NTHR>(
        NPART * nl * M,
        [&](int idx) {
            const int c = idx >> log2M;  // line: part c / nl, row c % nl
            const int64_t src = (c < nl ? row0 + c : row0 + (c - nl) + pair_offset);
            return Y[src * M + (idx & (M - 1))];
        },
        [&](int idx, c2<T> v) { buf[(idx >> log2M) * ld + padx(idx & (M - 1))] = v; });
    __syncthreads();
    irfft_unpack<T, NTHR>(buf, ld, NPART * nl, M, tw2);
    __syncthreads();
    lds_fft<T, NTHR, BPT>(buf, ld, NPART * nl, log2M, +1, twp);
    const int npair = n_out_cols / 2;
    double acc = 0.0;
    for (int c = 0; c < nl; ++c)
        for (int e = threadIdx.x; e < npair; e += NTHR) {
            const c2<T> z = buf[c * ld + padx(e)];
            const c2<T> w = NPART == 2 ? buf[(nl + c) * ld + padx(e)] : mk<T>(T(0), T(0));
            acc += epi(row0 + c, 2 * e, z.x, z.y, w.x, w.y);
        }
    acc = block_sum_n<NTHR>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Workgroups of launch_irfft_rows_pair for n_rows row pairs of packed width M.
inline int64_t irfft_pair_blocks(int M, int64_t n_rows, int npart, int n_cu, int *lpw_out, int *nthr_out) {
    int lpw = 1, nthr = 1024;
    if (npart * M <= 4096) {
        nthr = 256;
        lpw = std::max(1, 4096 / (npart * M));
        while (lpw > 1 && n_rows / lpw < 4 * (int64_t)std::max(n_cu, 1)) lpw >>= 1;
    }
    if (lpw_out) *lpw_out = lpw;
    if (nthr_out) *nthr_out = nthr;
    return (n_rows + lpw - 1) / lpw;
}

// Paired inverse row pass (power-of-two packed width M = 2^log2M <= 8192 / npart).
template <typename T, class Epi>
void launch_irfft_rows_pair(const Ctx &ctx, int log2M, int64_t n_rows, int64_t pair_offset, int npart,
                            int n_out_cols, Epi epi, const c2<T> *Y, double *partials, const int *skip,
                            hipStream_t st) {
    const int M = 1 << log2M;
    FR_REQUIRE(npart == 1 || npart == 2, "one or two images per pixel");
    FR_REQUIRE(npart * M <= 8192, "paired rows too long for one workgroup");
    int lpw = 1, nthr = 256;
    const int64_t nblk = irfft_pair_blocks(M, n_rows, npart, ctx.n_cu, &lpw, &nthr);
    const size_t lines = (size_t)npart * lpw * plen(M) * sizeof(c2<T>);
    const size_t twb = (size_t)M * sizeof(c2<T>);
    const c2<T> *tw = ctx.tw<T>(log2M), *tw2 = ctx.tw<T>(log2M + 1);
    FR_REQUIRE(lines <= (size_t)kLdsBytes, "paired rows exceed LDS");
    const bool twl = lines + twb <= (size_t)kLdsBytes;
    const size_t lds = twl ? lines + twb : lines;
#define FR_PAIR(NT, TW, NP)                                                                                   \
    do {                                                                                                      \
        allow_lds(k_irfft_rows_pair<T, NT, 4, TW, Epi, NP>, lds);                                             \
        k_irfft_rows_pair<T, NT, 4, TW, Epi, NP><<<dim3((unsigned)nblk), NT, lds, st>>>(                       \
            epi, Y, n_rows, pair_offset, log2M, n_out_cols, lpw, tw, tw2, partials, skip);                    \
    } while (0)
    if (nthr == 256) {
        if (npart == 2) FR_PAIR(256, true, 2);
        else FR_PAIR(256, true, 1);
    } else if (twl) {
        if (npart == 2) FR_PAIR(1024, true, 2);
        else FR_PAIR(1024, true, 1);
    } else {
        if (npart == 2) FR_PAIR(1024, false, 2);
        else FR_PAIR(1024, false, 1);
    }
#undef FR_PAIR
    LAUNCH_CHECK();
}

// ------------------------------------------------------------------ launchers
struct ConvGeom {
    int64_t n_img;   // images (each with its own kernel index g % nk)
    int rows_in;     // stored (non-zero) rows per image = n_in of the column pass
    int rows_out;    // rows kept after the column pass and written by pass 3
    int n_in_cols;   // non-zero real columns per row (<= 2M)
    int n_out_cols;  // real columns kept by pass 3
    int log2M;       // packed width M = odd_M 2^log2M
    int log2Lc;      // column FFT length Lc = odd_Lc 2^log2Lc
    int odd_M = 1, odd_Lc = 1;  // odd factors (1, 3 or 5) of M and Lc
    int M() const { return odd_M << log2M; }
    int Lc() const { return odd_Lc << log2Lc; }
};

template <typename T> inline int max_line_elems() { return kLdsBytes / (int)sizeof(c2<T>); }

// ODD must equal g.odd_M
template <typename T, int ODD = 1, class Pro>
void launch_rfft_rows(const Ctx &ctx, const ConvGeom &g, Pro pro, c2<T> *Y, hipStream_t st) {
    FR_REQUIRE(g.odd_M == ODD, "row length and kernel variant disagree");
    const int M = g.M();
    const int64_t nrows = g.n_img * g.rows_in;
    FR_REQUIRE(plen(M) <= max_line_elems<T>() && M <= 16384, "row length too large for LDS");
    const size_t line = (size_t)plen(M) * sizeof(c2<T>);
    const size_t twb = (size_t)M * sizeof(c2<T>);
    const c2<T> *tw = ctx.tw<T>(ODD, g.log2M), *tw2 = ctx.tw<T>(ODD, g.log2M + 1);
    if (M <= 4096) {
        const int lpw = rows_per_wg(M, nrows, ctx.n_cu);
        const int64_t nblk = (nrows + lpw - 1) / lpw;
        allow_lds(k_rfft_rows<T, 256, 4, true, Pro, ODD>, lpw * line + twb);
        k_rfft_rows<T, 256, 4, true, Pro, ODD><<<dim3((unsigned)nblk), 256, lpw * line + twb, st>>>(
            pro, Y, nrows, g.log2M, g.n_in_cols, lpw, tw, tw2);
    } else if (line + twb <= (size_t)kLdsBytes) {
        allow_lds(k_rfft_rows<T, 1024, 4, true, Pro, ODD>, line + twb);
        k_rfft_rows<T, 1024, 4, true, Pro, ODD><<<dim3((unsigned)nrows), 1024, line + twb, st>>>(
            pro, Y, nrows, g.log2M, g.n_in_cols, 1, tw, tw2);
    } else {
        allow_lds(k_rfft_rows<T, 1024, 4, false, Pro, ODD>, line);
        k_rfft_rows<T, 1024, 4, false, Pro, ODD><<<dim3((unsigned)nrows), 1024, line, st>>>(
            pro, Y, nrows, g.log2M, g.n_in_cols, 1, tw, tw2);
    }
    LAUNCH_CHECK();
}

// ODD must equal g.odd_Lc
template <typename T, int ODD = 1>
void launch_conv_cols(const Ctx &ctx, const ConvGeom &g, c2<T> *Y, const T *K, int nk, int mode, T scale,
                      hipStream_t st, const T *K_alt = nullptr, int64_t g_alt = INT64_MAX,
                      const int *skip = nullptr) {
    FR_REQUIRE(g.odd_Lc == ODD, "column length and kernel variant disagree");
    const int M = g.M();
    const int Lc = g.Lc();
    const int budget = 65536 / (int)sizeof(c2<T>);  // <= 64 KiB: two workgroups per CU
    const int cap = std::max(1, std::min(16, budget / Lc));
    int C = 1;
    while (2 * C <= cap) C *= 2;
    while (C > 1 && (M % C)) C >>= 1;
    // small batches: narrower strips so the grid still covers every CU a few times
    while (C > 2 && (int64_t)(M / C) * g.n_img < 2 * (int64_t)std::max(ctx.n_cu, 1)) C >>= 1;
    FR_REQUIRE((int64_t)C * (plen(Lc) + 1) <= max_line_elems<T>(), "column length too large for LDS");
    FR_REQUIRE(is_pow2(C), "column strip width must be a power of two");
    const size_t lds = (size_t)C * (plen(Lc) + 1) * sizeof(c2<T>);
    dim3 grid((unsigned)(M / C), (unsigned)g.n_img);
    FR_REQUIRE(g.rows_in == g.rows_out, "column pass works in place");
    const bool twl = lds + (size_t)Lc * sizeof(c2<T>) <= (size_t)kLdsBytes;
    const size_t ldst = twl ? lds + (size_t)Lc * sizeof(c2<T>) : lds;
#define FR_CONVCOLS(NT, TW)                                                                              \
    do {                                                                                                 \
        allow_lds(k_conv_cols<T, NT, 4, TW, ODD>, ldst);                                                 \
        k_conv_cols<T, NT, 4, TW, ODD><<<grid, NT, ldst, st>>>(Y, M, g.log2Lc, g.rows_in, g.rows_out, C, \
                                                               K, nk, mode, scale, ctx.tw<T>(ODD, g.log2Lc), \
                                                               K_alt, g_alt, skip);                          \
    } while (0)
    // one radix-4 butterfly per thread where the strip allows (the strip's load ->
    // FFT -> multiply -> FFT -> store chain is latency-bound; measured at
    // 512 x 512: batch 8, 8 columns: 1024 threads 15% faster than 512; batch 1,
    // 2 columns: 512 threads 16% faster than 256)
    if (C * Lc <= 1024) {
        if (twl) FR_CONVCOLS(256, true);
        else FR_CONVCOLS(256, false);
    } else if (C * Lc <= 2048) {
        if (twl) FR_CONVCOLS(512, true);
        else FR_CONVCOLS(512, false);
    } else {
        if (twl) FR_CONVCOLS(1024, true);
        else FR_CONVCOLS(1024, false);
    }
#undef FR_CONVCOLS
    LAUNCH_CHECK();
}

// ODD must equal g.odd_M
template <typename T, int ODD = 1, class Epi>
void launch_irfft_rows(const Ctx &ctx, const ConvGeom &g, Epi epi, const c2<T> *Y, hipStream_t st) {
    FR_REQUIRE(g.odd_M == ODD, "row length and kernel variant disagree");
    const int M = g.M();
    const int64_t nrows = g.n_img * g.rows_out;
    const size_t line = (size_t)plen(M) * sizeof(c2<T>);
    const size_t twb = (size_t)M * sizeof(c2<T>);
    const c2<T> *tw = ctx.tw<T>(ODD, g.log2M), *tw2 = ctx.tw<T>(ODD, g.log2M + 1);
    if (M <= 4096) {
        const int lpw = rows_per_wg(M, nrows, ctx.n_cu);
        const int64_t nblk = (nrows + lpw - 1) / lpw;
        allow_lds(k_irfft_rows<T, 256, 4, true, Epi, ODD>, lpw * line + twb);
        k_irfft_rows<T, 256, 4, true, Epi, ODD><<<dim3((unsigned)nblk), 256, lpw * line + twb, st>>>(
            epi, Y, nrows, g.log2M, g.n_out_cols, lpw, tw, tw2);
    } else if (line + twb <= (size_t)kLdsBytes) {
        allow_lds(k_irfft_rows<T, 1024, 4, true, Epi, ODD>, line + twb);
        k_irfft_rows<T, 1024, 4, true, Epi, ODD><<<dim3((unsigned)nrows), 1024, line + twb, st>>>(
            epi, Y, nrows, g.log2M, g.n_out_cols, 1, tw, tw2);
    } else {
        allow_lds(k_irfft_rows<T, 1024, 4, false, Epi, ODD>, line);
        k_irfft_rows<T, 1024, 4, false, Epi, ODD><<<dim3((unsigned)nrows), 1024, line, st>>>(
            epi, Y, nrows, g.log2M, g.n_out_cols, 1, tw, tw2);
    }
    LAUNCH_CHECK();
}

// ------------------------------------------------------------------ functors
// (nx is a power of two: row % nx is row & (nx - 1); rows stay below 2^31)
// x[q] * d[q] * a[row % nx][col] with optional full-size d and per-pixel a (q = row * ny + col)
template <typename T> struct ProDiagScaled {
    const T *x, *d, *a;
    int nx, ny;
    __device__ T operator()(int64_t row, int col) const {
        const int64_t q = row * ny + col;
        T v = x[q];
        if (d) v *= d[q];
        if (a) v *= a[((int)row & (nx - 1)) * ny + col];
        return v;
    }
};

// y[q] = d[q] * a[row % nx][col] * value + add[q]
template <typename T> struct EpiDiagScaledAdd {
    T *y;
    const T *d, *a, *add;
    int nx, ny;
    __device__ void operator()(int64_t row, int col, T v0, T v1) const {
        const int64_t q = row * ny + col;
        if (d) {
            v0 *= d[q];
            v1 *= d[q + 1];
        }
        if (a) {
            const T *pa = a + ((int)row & (nx - 1)) * ny + col;
            v0 *= pa[0];
            v1 *= pa[1];
        }
        if (add) {
            v0 += add[q];
            v1 += add[q + 1];
        }
        y[q] = v0;
        y[q + 1] = v1;
    }
};

}  // namespace frmi
