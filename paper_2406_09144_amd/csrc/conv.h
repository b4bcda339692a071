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


// ------------------------------------------------------------------ pass 2, long columns
// For columns of L = L1 L2 points (L >= 8192) a strip of a few columns no longer
// fits the LDS, and single-column strips read each row with one isolated 8-byte
// access.  The column convolution then runs as a four-step FFT over strips of C
// adjacent columns (one row access moves C values), through a scratch Z of L rows:
//   step 1: for each n2 < L2, the L1-point FFTs of x[L2 n1 + n2] over n1 (strided
//           rows), times exp(-2 pi i n2 k1 / L), into Z row L2 k1 + n2;
//   step 2: for each k1 < L1, the L2-point FFT of Z rows L2 k1 + (0 .. L2-1) gives
//           X[k1 + L1 k2] at row L2 k1 + k2; multiply by the kernel at frequency
//           k1 + L1 k2; the inverse L2-point FFT over k2 and exp(+2 pi i m2 k1 / L)
//           give the partial inverse at row L2 k1 + m2;
//   step 3: for each m2 < L2, the inverse L1-point FFT over k1 of the rows
//           L2 k1 + m2 gives y[L2 m1 + m2], of which rows < n_out are stored.
// The packed column 0 (DC and Nyquist columns, whose kernel multiply needs the
// mirrored frequency -k) is left to the single-column kernel.
// Thread layout of a load or store: column fastest (C values of a row), then the
// group member (adjacent rows in steps 1 and 3), then the element along the line.
template <typename T, int NTHR, int BPT>
__global__ __launch_bounds__(NTHR) void k_conv4_outer(const c2<T> *__restrict__ src, int64_t src_rows_img,
                                                       c2<T> *__restrict__ dst, int64_t dst_rows_img, int M,
                                                       int log2L1, int log2L2, int n_valid_src, int n_valid_dst,
                                                       int log2C, int log2G, int sign, int skip_col0,
                                                       const c2<T> *__restrict__ tw1,
                                                       const c2<T> *__restrict__ twL,
                                                       const int *__restrict__ skip) {
    if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int L1 = 1 << log2L1, L2 = 1 << log2L2, C = 1 << log2C, G = 1 << log2G;
    const int ld = plen(L1) + 1;
    const int nlines = C * G;
    const int col0 = blockIdx.x << log2C;
    const int n2_0 = blockIdx.y << log2G;
    const int64_t img = blockIdx.z;
    const c2<T> *S = src + img * src_rows_img * (int64_t)M;
    c2<T> *D = dst + img * dst_rows_img * (int64_t)M;
    const int log2L = log2L1 + log2L2;
    // the forward pass's split twiddles exp(-2 pi i n2 k1 / L) of this thread's
    // stores, fetched before the line loads so that they arrive during the FFT
    // (a load inside the store loop would put one memory round trip per element
    // on the thread's critical path)
    constexpr int EPT = 4 * BPT;  // elements per thread: nlines L1 <= 4 BPT NTHR
    c2<T> twr[EPT];
    if (sign < 0) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int idx = threadIdx.x + j * NTHR;
            const int gg = (idx >> log2C) & (G - 1), k1 = idx >> (log2C + log2G);
            twr[j] = idx < nlines * L1 ? twL[((n2_0 + gg) * k1) & ((1 << log2L) - 1)] : mk<T>(T(1), T(0));
        }
    }
    const c2<T> *twp = stage_twiddles<T, NTHR, true>(buf + nlines * ld, tw1, L1);
    // load: element n1 of line (g, c) is row L2 n1 + n2_0 + g of column col0 + c
    staged_copy<NTHR>(
        nlines * L1,
        [&](int idx) {
            const int c = idx & (C - 1), gg = (idx >> log2C) & (G - 1), n1 = idx >> (log2C + log2G);
            const int r = (n1 << log2L2) + n2_0 + gg;
            return r < n_valid_src ? S[(int64_t)r * M + col0 + c] : mk<T>(T(0), T(0));
        },
        [&](int idx, c2<T> v) {
            const int c = idx & (C - 1), gg = (idx >> log2C) & (G - 1), n1 = idx >> (log2C + log2G);
            buf[(gg * C + c) * ld + padx(n1)] = v;
        });
    __syncthreads();
    lds_fft<T, NTHR, BPT, 1, kFixAll>(buf, ld, nlines, log2L1, sign, twp);
    // store: element k1 of line (g, c) to row L2 k1 + n2 (forward: times the twiddle
    // exp(-2 pi i n2 k1 / L) of the four-step split)
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int idx = threadIdx.x + j * NTHR;
        if (idx >= nlines * L1) break;
        const int c = idx & (C - 1), gg = (idx >> log2C) & (G - 1), k1 = idx >> (log2C + log2G);
        const int r = (k1 << log2L2) + n2_0 + gg;
        if (r >= n_valid_dst || (skip_col0 && col0 + c == 0)) continue;
        c2<T> v = buf[(gg * C + c) * ld + padx(k1)];
        if (sign < 0) v = cmul<T>(v, twr[j]);
        D[(int64_t)r * M + col0 + c] = v;
    }
}

// step 2: for k1 in this workgroup's group, forward L2-point FFT, kernel multiply,
// inverse L2-point FFT, inverse twiddle; in place on Z.
template <typename T, int NTHR, int BPT>
__global__ __launch_bounds__(NTHR) void k_conv4_middle(c2<T> *__restrict__ Z, int64_t z_rows_img, int M,
                                                        int log2L1, int log2L2, int log2C, int log2G,
                                                        const T *__restrict__ K, int nk, int mode, T scale,
                                                        const c2<T> *__restrict__ tw2,
                                                        const c2<T> *__restrict__ twL,
                                                        const T *__restrict__ K_alt, int64_t g_alt,
                                                        const int *__restrict__ skip) {
    if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int L1 = 1 << log2L1, L2 = 1 << log2L2, C = 1 << log2C, G = 1 << log2G;
    const int L = L1 * L2;
    const int ld = plen(L2) + 1;
    const int nlines = C * G;
    const int col0 = blockIdx.x << log2C;
    const int k1_0 = blockIdx.y << log2G;
    const int64_t img = blockIdx.z;
    c2<T> *Zi = Z + img * z_rows_img * (int64_t)M;
    const T *Kg = img >= g_alt ? K_alt : K + (img % nk) * (int64_t)L * (M + 1);
    // this thread's kernel values, fetched before the line loads so that they
    // arrive during the forward FFT (element idx = threadIdx.x + j NTHR: column
    // fastest, then the element k2 (or m2) along the line, then the group member)
    constexpr int EPT = 4 * BPT;  // nlines L2 <= 4 BPT NTHR
    T kr[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int idx = threadIdx.x + j * NTHR;
        const int c = idx & (C - 1), e = (idx >> log2C) & (L2 - 1), gg = idx >> (log2C + log2L2);
        kr[j] = idx < nlines * L2 ? Kg[(int64_t)((k1_0 + gg) + (e << log2L1)) * (M + 1) + col0 + c] : T(0);
    }
    const c2<T> *twp = stage_twiddles<T, NTHR, true>(buf + nlines * ld, tw2, L2);
    auto row_of = [&](int gg, int e) { return ((k1_0 + gg) << log2L2) + e; };
    staged_copy<NTHR>(
        nlines * L2,
        [&](int idx) {
            const int c = idx & (C - 1), e = (idx >> log2C) & (L2 - 1), gg = idx >> (log2C + log2L2);
            return Zi[(int64_t)row_of(gg, e) * M + col0 + c];
        },
        [&](int idx, c2<T> v) {
            const int c = idx & (C - 1), e = (idx >> log2C) & (L2 - 1), gg = idx >> (log2C + log2L2);
            buf[(gg * C + c) * ld + padx(e)] = v;
        });
    __syncthreads();
    lds_fft<T, NTHR, BPT, 1, kFixAll>(buf, ld, nlines, log2L2, -1, twp);
    // the inverse split twiddles of this thread's stores, in flight during the
    // multiply and the inverse FFT
    c2<T> twr[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int idx = threadIdx.x + j * NTHR;
        const int e = (idx >> log2C) & (L2 - 1), gg = idx >> (log2C + log2L2);
        twr[j] = idx < nlines * L2 ? twL[(e * (k1_0 + gg)) & (L - 1)] : mk<T>(T(1), T(0));
    }
    // element k2 of line (g, c) holds frequency k = k1 + L1 k2 of column col0 + c
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int idx = threadIdx.x + j * NTHR;
        if (idx >= nlines * L2) break;
        const int c = idx & (C - 1), k2 = (idx >> log2C) & (L2 - 1), gg = idx >> (log2C + log2L2);
        const T kv = kernel_factor(kr[j], mode) * scale;
        c2<T> &v = buf[(gg * C + c) * ld + padx(k2)];
        v = mk<T>(v.x * kv, v.y * kv);
    }
    __syncthreads();
    lds_fft<T, NTHR, BPT, 1, kFixAll>(buf, ld, nlines, log2L2, +1, twp);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int idx = threadIdx.x + j * NTHR;
        if (idx >= nlines * L2) break;
        const int c = idx & (C - 1), m2 = (idx >> log2C) & (L2 - 1), gg = idx >> (log2C + log2L2);
        const c2<T> v = buf[(gg * C + c) * ld + padx(m2)];
        const c2<T> w = cconj<T>(twr[j]);  // exp(+2 pi i m2 k1 / L)
        Zi[(int64_t)row_of(gg, m2) * M + col0 + c] = cmul<T>(v, w);
    }
}

// Columns per strip and group sizes of the four-step column pass (C columns of
// 8 or 16 bytes: 128-byte row segments; G lines per workgroup so that C G L_i is
// 4096 elements, one radix-16 butterfly per thread of 256).
inline void conv4_shape(int log2L, int M, int esize, int *log2L1, int *log2L2, int *log2C, int *log2G1,
                        int *log2G2) {
    *log2L1 = log2L / 2;
    *log2L2 = log2L - *log2L1;
    int lc = esize == 8 ? 4 : 3;  // 16 or 8 columns: 128 bytes
    while (lc > 0 && (M % (1 << lc))) --lc;
    *log2C = lc;
    *log2G1 = std::max(0, 12 - *log2L1 - lc);
    *log2G2 = std::max(0, 12 - *log2L2 - lc);
    *log2G1 = std::min(*log2G1, *log2L2);  // groups of n2 < L2
    *log2G2 = std::min(*log2G2, *log2L1);  // groups of k1 < L1
}

inline bool conv4_applies(int Lc, int odd, int M, size_t esize) {
    return odd == 1 && Lc >= 8192 && M >= 8 && M % 2 == 0 && (esize == 8 || esize == 16);
}

// scratch of the four-step pass: L rows of M complex values per image
inline size_t conv4_scratch(int64_t n_img, int Lc, int M, size_t csize) {
    return (size_t)n_img * Lc * M * csize;
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

// Several FP64 sums carried together (an epilogue may return one of these
// instead of a double to contribute to N sums at once).
template <int N> struct SumN {
    double v[N];
};
template <class R> struct sum_count { static constexpr int n = 1; };
template <int N> struct sum_count<SumN<N>> { static constexpr int n = N; };
template <int N> __device__ __forceinline__ void sum_add(double (&acc)[N], const SumN<N> &x) {
#pragma unroll
    for (int j = 0; j < N; ++j) acc[j] += x.v[j];
}
__device__ __forceinline__ void sum_add(double (&acc)[1], double x) { acc[0] += x; }

// Pass 3 over pairs of images: row r of the first n_rows packed rows goes with
// row r + pair_offset (NPART = 2; NPART = 1 has no partner), both inverse
// transformed in the same workgroup so that the epilogue sees the two real
// values of a pixel together: epi(r, col, a0, a1, b0, b1) receives columns col
// and col + 1 of the row and of its partner, stores what it needs and returns a
// contribution to a sum (a double) or to N sums (SumN<N>); the workgroup's FP64
// sums go to partials[blockIdx.x * N + j].  A non-zero *skip turns the launch
// into a no-op.
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
    constexpr int NS = sum_count<decltype(epi(int64_t(0), 0, T(0), T(0), T(0), T(0)))>::n;
    double acc[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) acc[j] = 0.0;
    for (int c = 0; c < nl; ++c)
        for (int e = threadIdx.x; e < npair; e += NTHR) {
            const c2<T> z = buf[c * ld + padx(e)];
            const c2<T> w = NPART == 2 ? buf[(nl + c) * ld + padx(e)] : mk<T>(T(0), T(0));
            sum_add(acc, epi(row0 + c, 2 * e, z.x, z.y, w.x, w.y));
        }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const double t = block_sum_n<NTHR>(acc[j]);
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * NS + j] = t;
    }
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

// Row passes keep the twiddle table in LDS only while it is at most half the
// lines' size: a 4096-point line (lines and table of about 33 KB each) then runs
// four workgroups per CU instead of two (4096^2 PSF apply, 16 images: both row
// passes 1.7 -> 1.25-1.3 ms)
inline bool twl_small(size_t line_bytes, size_t tw_bytes) { return 2 * tw_bytes <= line_bytes; }

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
        if (twl_small(lpw * line, twb)) {
            allow_lds(k_rfft_rows<T, 256, 4, true, Pro, ODD>, lpw * line + twb);
            k_rfft_rows<T, 256, 4, true, Pro, ODD><<<dim3((unsigned)nblk), 256, lpw * line + twb, st>>>(
                pro, Y, nrows, g.log2M, g.n_in_cols, lpw, tw, tw2);
        } else {
            allow_lds(k_rfft_rows<T, 256, 4, false, Pro, ODD>, lpw * line);
            k_rfft_rows<T, 256, 4, false, Pro, ODD><<<dim3((unsigned)nblk), 256, lpw * line, st>>>(
                pro, Y, nrows, g.log2M, g.n_in_cols, lpw, tw, tw2);
        }
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

// Scratch bytes of the column pass beyond Y: the four-step path's Z, else 0.
template <typename T> inline size_t conv_cols_scratch(const ConvGeom &g) {
    return conv4_applies(g.Lc(), g.odd_Lc, g.M(), sizeof(c2<T>))
               ? conv4_scratch(g.n_img, g.Lc(), g.M(), sizeof(c2<T>))
               : 0;
}

// Four-step column convolution of long power-of-two columns (see k_conv4_outer);
// Z: conv_cols_scratch bytes, from the stream's arena when null.
template <typename T>
void launch_conv_cols_4step(const Ctx &ctx, const ConvGeom &g, c2<T> *Y, const T *K, int nk, int mode, T scale,
                            hipStream_t st, const T *K_alt, int64_t g_alt, const int *skip, void *zws) {
    const int M = g.M();
    const int Lc = g.Lc();
    int l1, l2, lc, lg1, lg2;
    conv4_shape(g.log2Lc, M, (int)sizeof(c2<T>), &l1, &l2, &lc, &lg1, &lg2);
    FR_REQUIRE(lc >= 1 && (M % (1 << lc)) == 0, "four-step column pass needs an even packed width");
    FR_REQUIRE(g.n_img <= 65535, "too many images for one column pass");
    FR_REQUIRE(g.rows_in == g.rows_out && g.rows_in <= Lc, "column pass works in place");
    // the packed column 0 (DC and Nyquist columns) first, by the strip kernel with
    // one single-column strip per image: it reads and writes column 0 of Y only,
    // which the last four-step pass leaves alone
    {
        const int ld = plen(Lc) + 1;
        const size_t lds = (size_t)ld * sizeof(c2<T>);
        const bool twl = lds + (size_t)Lc * sizeof(c2<T>) <= (size_t)kLdsBytes;
        FR_REQUIRE(lds <= (size_t)kLdsBytes, "column length too large for LDS");
        const dim3 grid0(1u, (unsigned)g.n_img);
        if (twl) {
            const size_t b = lds + (size_t)Lc * sizeof(c2<T>);
            allow_lds(k_conv_cols<T, 1024, 4, true, 1>, b);
            k_conv_cols<T, 1024, 4, true, 1><<<grid0, 1024, b, st>>>(Y, M, g.log2Lc, g.rows_in, g.rows_out, 1, K,
                                                                     nk, mode, scale, ctx.tw<T>(g.log2Lc), K_alt,
                                                                     g_alt, skip);
        } else {
            allow_lds(k_conv_cols<T, 1024, 4, false, 1>, lds);
            k_conv_cols<T, 1024, 4, false, 1><<<grid0, 1024, lds, st>>>(Y, M, g.log2Lc, g.rows_in, g.rows_out, 1,
                                                                        K, nk, mode, scale, ctx.tw<T>(g.log2Lc),
                                                                        K_alt, g_alt, skip);
        }
        LAUNCH_CHECK();
    }
    Scratch Zarena;
    if (!zws) Zarena = Scratch(conv4_scratch(g.n_img, Lc, M, sizeof(c2<T>)), st);
    c2<T> *const Z = zws ? (c2<T> *)zws : Zarena.as<c2<T>>();
    const int L1 = 1 << l1, L2 = 1 << l2, C = 1 << lc;
    const size_t lds1 = ((size_t)(C << lg1) * (plen(L1) + 1) + L1) * sizeof(c2<T>);
    const size_t lds2 = ((size_t)(C << lg2) * (plen(L2) + 1) + L2) * sizeof(c2<T>);
    const dim3 grid1((unsigned)(M / C), (unsigned)(L2 >> lg1), (unsigned)g.n_img);
    const dim3 grid2((unsigned)(M / C), (unsigned)(L1 >> lg2), (unsigned)g.n_img);
    const c2<T> *twL = ctx.tw<T>(g.log2Lc);
    allow_lds(k_conv4_outer<T, 256, 4>, lds1);
    allow_lds(k_conv4_middle<T, 256, 4>, lds2);
    k_conv4_outer<T, 256, 4><<<grid1, 256, lds1, st>>>(Y, g.rows_in, Z, Lc, M, l1, l2, g.rows_in, Lc, lc, lg1, -1, 0,
                                                       ctx.tw<T>(l1), twL, skip);
    LAUNCH_CHECK();
    k_conv4_middle<T, 256, 4><<<grid2, 256, lds2, st>>>(Z, Lc, M, l1, l2, lc, lg2, K, nk, mode, scale,
                                                        ctx.tw<T>(l2), twL, K_alt, g_alt, skip);
    LAUNCH_CHECK();
    k_conv4_outer<T, 256, 4><<<grid1, 256, lds1, st>>>(Z, Lc, Y, g.rows_out, M, l1, l2, Lc, g.rows_out, lc, lg1, +1, 1,
                                                       ctx.tw<T>(l1), twL, skip);
    LAUNCH_CHECK();
}

// ODD must equal g.odd_Lc.  zws: conv_cols_scratch bytes (only the four-step path
// of long columns uses it), from the stream's arena when null.
template <typename T, int ODD = 1>
void launch_conv_cols(const Ctx &ctx, const ConvGeom &g, c2<T> *Y, const T *K, int nk, int mode, T scale,
                      hipStream_t st, const T *K_alt = nullptr, int64_t g_alt = INT64_MAX,
                      const int *skip = nullptr, void *zws = nullptr) {
    FR_REQUIRE(g.odd_Lc == ODD, "column length and kernel variant disagree");
    const int M = g.M();
    const int Lc = g.Lc();
    if (conv4_applies(Lc, ODD, M, sizeof(c2<T>))) {
        launch_conv_cols_4step<T>(ctx, g, Y, K, nk, mode, scale, st, K_alt, g_alt, skip, zws);
        return;
    }
    const int budget = 65536 / (int)sizeof(c2<T>);  // <= 64 KiB: two workgroups per CU
    const int cap = std::max(1, std::min(16, budget / Lc));
    int C = 1;
    while (2 * C <= cap) C *= 2;
    while (C > 1 && (M % C)) C >>= 1;
    // small batches: narrower strips so the grid still covers every CU a few times
    while (C > 2 && (int64_t)(M / C) * g.n_img < 2 * (int64_t)std::max(ctx.n_cu, 1)) C >>= 1;
    // long columns (one line already fills 64 KiB): strips of two columns, so that
    // each row access moves two adjacent values, at one workgroup per CU
    if (C == 1 && M % 2 == 0 && (int64_t)2 * (plen(Lc) + 1) <= max_line_elems<T>()) C = 2;
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
        if (twl_small(lpw * line, twb)) {
            allow_lds(k_irfft_rows<T, 256, 4, true, Epi, ODD>, lpw * line + twb);
            k_irfft_rows<T, 256, 4, true, Epi, ODD><<<dim3((unsigned)nblk), 256, lpw * line + twb, st>>>(
                epi, Y, nrows, g.log2M, g.n_out_cols, lpw, tw, tw2);
        } else {
            allow_lds(k_irfft_rows<T, 256, 4, false, Epi, ODD>, lpw * line);
            k_irfft_rows<T, 256, 4, false, Epi, ODD><<<dim3((unsigned)nblk), 256, lpw * line, st>>>(
                epi, Y, nrows, g.log2M, g.n_out_cols, lpw, tw, tw2);
        }
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
