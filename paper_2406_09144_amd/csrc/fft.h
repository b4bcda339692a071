// Stockham FFT on LDS-resident lines, shared by every transform in the library
// (uv-grid FFTs of the gridder, the zero-padded PSF convolution, the periodic
// noise and prior convolutions).
//
// Method: the self-sorting Stockham formulation (natural-order output without a
// bit-reversal pass) of Govindaraju et al., "High performance discrete Fourier
// transforms on graphics processors" (SC'08).  A stage with current span Ns and
// radix R takes, for every butterfly index j < L/R with k = j mod Ns,
//   v_r = x[j + r L/R] * exp(sign 2 pi i r k / (Ns R)),  r < R,
// applies the R-point DFT, and writes y[(j / Ns) Ns R + k + r Ns] = v_r.
// Lines live in LDS; each butterfly keeps its R values in registers between the
// read and the write barrier, so a stage is in place.
//
// Lengths are L = ODD 2^p with ODD in {1, 3, 5}: radix-16, 4 and 2 stages take
// the power of two, then one radix-ODD stage (Ns = 2^p) the odd factor, so Ns
// stays a power of two throughout and only the butterfly-to-line split divides
// by ODD.  The odd lengths serve the reduced zero padding of the PSF
// convolution (n + h instead of 2n).
//
// Twiddles come from a per-length table tw[m] = exp(-2 pi i m / L) built in FP64
// on the host and rounded once to the working precision.
#pragma once

#include "common.h"

namespace frmi {

// LDS lines are padded by one element after every 32 (element e of a line at
// padx(e)), so that the strided stores of the early Stockham stages and the
// transposed strip accesses spread over the banks.
__host__ __device__ constexpr int padx(int e) { return e + (e >> 5); }
__host__ __device__ constexpr int plen(int L) { return L + (L >> 5); }

// The transform direction SIGN (-1 forward, +1 inverse) is a template argument
// throughout, so the quarter turns, the internal rotations and the twiddle
// conjugation compile to plain operand swaps and sign modifiers.
template <typename T, int SIGN>
__device__ __forceinline__ c2<T> mul_i_sign(c2<T> a) {
    // a * (SIGN * i)
    if constexpr (SIGN < 0) return mk<T>(a.y, -a.x);
    else return mk<T>(-a.y, a.x);
}

template <typename T>
__device__ __forceinline__ void dft2(c2<T> (&v)[2]) {
    c2<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
}

template <typename T, int SIGN>
__device__ __forceinline__ void dft4(c2<T> (&v)[4]) {
    c2<T> t0 = cadd<T>(v[0], v[2]);
    c2<T> t1 = csub<T>(v[0], v[2]);
    c2<T> t2 = cadd<T>(v[1], v[3]);
    c2<T> t3 = mul_i_sign<T, SIGN>(csub<T>(v[1], v[3]));
    v[0] = cadd<T>(t0, t2);
    v[2] = csub<T>(t0, t2);
    v[1] = cadd<T>(t1, t3);
    v[3] = csub<T>(t1, t3);
}

// v * exp(SIGN 2 pi i M / 16), M < 16, from the exact values of cos and sin at
// multiples of pi / 8
template <typename T, int SIGN, int M>
__device__ __forceinline__ c2<T> rot16(c2<T> v) {
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, r2 = 0.70710678118654752440;
    constexpr double cs[5] = {1.0, c1, r2, s1, 0.0};  // cos(r pi / 8), r = 0..4
    constexpr int q = M >> 2, r = M & 3;              // M pi / 8 = q pi / 2 + r pi / 8
    c2<T> w = v;
    if constexpr (r != 0) {
        constexpr T c = (T)cs[r], sn = (T)(SIGN * cs[4 - r]);  // cos and SIGN sin of r pi / 8
        w = mk<T>(v.x * c - v.y * sn, v.y * c + v.x * sn);
    }
    if constexpr (q >= 1) w = mul_i_sign<T, SIGN>(w);
    if constexpr (q >= 2) w = mul_i_sign<T, SIGN>(w);
    if constexpr (q >= 3) w = mul_i_sign<T, SIGN>(w);
    return w;
}

template <typename T, int SIGN, int N2>
__device__ __forceinline__ void dft16_col(c2<T> (&v)[16], c2<T> (&a)[4][4]) {
    c2<T> t[4] = {v[N2], v[4 + N2], v[8 + N2], v[12 + N2]};
    dft4<T, SIGN>(t);
    a[N2][0] = t[0];
    a[N2][1] = rot16<T, SIGN, N2 * 1>(t[1]);
    a[N2][2] = rot16<T, SIGN, N2 * 2>(t[2]);
    a[N2][3] = rot16<T, SIGN, N2 * 3>(t[3]);
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2,
//   X[k1 + 4 k2] = sum_n2 W16^(n2 k1) W4^(n2 k2) sum_n1 x[4 n1 + n2] W4^(n1 k1)
template <typename T, int SIGN>
__device__ __forceinline__ void dft16(c2<T> (&v)[16]) {
    c2<T> a[4][4];
    dft16_col<T, SIGN, 0>(v, a);
    dft16_col<T, SIGN, 1>(v, a);
    dft16_col<T, SIGN, 2>(v, a);
    dft16_col<T, SIGN, 3>(v, a);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        c2<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<T, SIGN>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
}

// 3-point DFT: w = exp(SIGN 2 pi i / 3) = -1/2 + SIGN i sqrt(3)/2, so
//   X1, X2 = a - (b + c)/2 +- SIGN i (sqrt(3)/2)(b - c)
template <typename T, int SIGN>
__device__ __forceinline__ void dft3(c2<T> (&v)[3]) {
    constexpr double h3 = 0.86602540378443864676;  // sqrt(3) / 2
    const c2<T> s = cadd<T>(v[1], v[2]);
    const c2<T> m = mk<T>(v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y);
    const c2<T> d = mul_i_sign<T, SIGN>(cscale<T>(csub<T>(v[1], v[2]), T(h3)));
    v[0] = cadd<T>(v[0], s);
    v[1] = cadd<T>(m, d);
    v[2] = csub<T>(m, d);
}

// 5-point DFT from the pairs A_r = x_r + x_{5-r}, B_r = x_r - x_{5-r} (r = 1, 2):
//   X1, X4 = x0 + c1 A1 + c2 A2 +- SIGN i (s1 B1 + s2 B2)
//   X2, X3 = x0 + c2 A1 + c1 A2 +- SIGN i (s2 B1 - s1 B2)
// with c_r = cos(2 pi r / 5), s_r = sin(2 pi r / 5).
template <typename T, int SIGN>
__device__ __forceinline__ void dft5(c2<T> (&v)[5]) {
    constexpr double c1 = 0.30901699437494742410, c2_ = -0.80901699437494742410;
    constexpr double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    const c2<T> A1 = cadd<T>(v[1], v[4]), B1 = csub<T>(v[1], v[4]);
    const c2<T> A2 = cadd<T>(v[2], v[3]), B2 = csub<T>(v[2], v[3]);
    const c2<T> e1 = mk<T>(v[0].x + T(c1) * A1.x + T(c2_) * A2.x, v[0].y + T(c1) * A1.y + T(c2_) * A2.y);
    const c2<T> e2 = mk<T>(v[0].x + T(c2_) * A1.x + T(c1) * A2.x, v[0].y + T(c2_) * A1.y + T(c1) * A2.y);
    const c2<T> o1 = mul_i_sign<T, SIGN>(mk<T>(T(s1) * B1.x + T(s2) * B2.x, T(s1) * B1.y + T(s2) * B2.y));
    const c2<T> o2 = mul_i_sign<T, SIGN>(mk<T>(T(s2) * B1.x - T(s1) * B2.x, T(s2) * B1.y - T(s1) * B2.y));
    v[0] = cadd<T>(v[0], cadd<T>(A1, A2));
    v[1] = cadd<T>(e1, o1);
    v[4] = csub<T>(e1, o1);
    v[2] = cadd<T>(e2, o2);
    v[3] = csub<T>(e2, o2);
}

template <typename T, int R, int SIGN>
__device__ __forceinline__ void dftR(c2<T> (&v)[R]) {
    if constexpr (R == 2) dft2<T>(v);
    else if constexpr (R == 3) dft3<T, SIGN>(v);
    else if constexpr (R == 4) dft4<T, SIGN>(v);
    else if constexpr (R == 5) dft5<T, SIGN>(v);
    else dft16<T, SIGN>(v);
}

// x / ODD for x >= 0 (a multiply-high for ODD = 3, 5; nothing for ODD = 1)
template <int ODD> __device__ __forceinline__ int div_odd(int x) {
    if constexpr (ODD == 1) return x;
    else return (int)((unsigned)x / (unsigned)ODD);
}

// One Stockham stage over `nlines` lines of length L = ODD 2^log2P spaced `ld`
// apart.  R is 16, 4 or 2 (a power-of-two stage, Ns = 2^log2Ns) or R = ODD (the
// final odd stage, Ns = 2^log2P).
// BPT: butterflies per thread this launch can need (host-checked).
template <typename T, int R, int NTHR, int BPT, int ODD, int SIGN>
__device__ __forceinline__ void stockham_stage(c2<T> *buf, int ld, int nlines, int log2P, int log2Ns,
                                               const c2<T> *__restrict__ tw) {
    constexpr bool kOddStage = (R == 3 || R == 5);
    static_assert(!kOddStage || R == ODD, "the odd stage takes the odd factor of the length");
    constexpr int LOG2R = kOddStage ? 0 : (R == 2) ? 1 : (R == 4) ? 2 : 4;
    // Q = L / R butterflies per line: QODD 2^log2Qp; twiddle stride L / (Ns R) = QODD 2^twshift
    constexpr int QODD = kOddStage ? 1 : ODD;
    const int log2Qp = log2P - LOG2R;
    const int Q = QODD << log2Qp;
    const int nb = nlines * Q;
    const int Ns = 1 << log2Ns;
    const int twshift = log2P - log2Ns - LOG2R;
    c2<T> v[BPT][R];
    int obase[BPT];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int f = threadIdx.x + b * NTHR;
        obase[b] = -1;
        if (f < nb) {
            const int line = div_odd<QODD>(f >> log2Qp);
            const int j = (QODD == 1) ? (f & (Q - 1)) : f - line * Q;
            const int k = j & (Ns - 1);
            const c2<T> *p = buf + line * ld;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = p[padx(j + r * Q)];
            if (log2Ns > 0) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    c2<T> w = tw[(r * k * QODD) << twshift];
                    if constexpr (SIGN > 0) w.y = -w.y;
                    v[b][r] = cmul<T>(v[b][r], w);
                }
            }
            dftR<T, R, SIGN>(v[b]);
            obase[b] = (line << 16) | (((j >> log2Ns) << (log2Ns + LOG2R)) + k);  // line, element
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        if (obase[b] >= 0) {
            c2<T> *p = buf + (obase[b] >> 16) * ld;
            const int e0 = obase[b] & 0xffff;
#pragma unroll
            for (int r = 0; r < R; ++r) p[padx(e0 + r * Ns)] = v[b][r];
        }
    }
    __syncthreads();
}

// Full in-place FFT of `nlines` LDS lines (length L = ODD 2^log2P <= 16384,
// stride ld >= plen(L), element e at padx(e); nlines < 32768).  Caller must
// __syncthreads() after filling the lines; returns after a barrier.
// Requires nlines * L <= 4 * BPT * NTHR.
template <typename T, int NTHR, int BPT, int ODD, int SIGN>
__device__ __forceinline__ void lds_fft_dir(c2<T> *buf, int ld, int nlines, int log2P,
                                            const c2<T> *__restrict__ tw) {
    static_assert(ODD == 1 || ODD == 3 || ODD == 5, "line lengths are 2^p, 3 2^p or 5 2^p");
    // radix-16 stages (two radix-4 levels in registers, half the LDS passes),
    // then radix 4 and 2 for the remaining power of two, then the odd factor
    constexpr int BPT16 = BPT / 4 > 0 ? BPT / 4 : 1;
    int log2Ns = 0;
    while (log2P - log2Ns >= 4) {
        stockham_stage<T, 16, NTHR, BPT16, ODD, SIGN>(buf, ld, nlines, log2P, log2Ns, tw);
        log2Ns += 4;
    }
    if (log2P - log2Ns >= 2) {
        stockham_stage<T, 4, NTHR, BPT, ODD, SIGN>(buf, ld, nlines, log2P, log2Ns, tw);
        log2Ns += 2;
    }
    if (log2P - log2Ns == 1) stockham_stage<T, 2, NTHR, 2 * BPT, ODD, SIGN>(buf, ld, nlines, log2P, log2Ns, tw);
    if constexpr (ODD > 1)
        stockham_stage<T, ODD, NTHR, (4 * BPT + ODD - 1) / ODD, ODD, SIGN>(buf, ld, nlines, log2P, log2P, tw);
}

// The same stage for a power-of-two length 2^LOG2P fixed at compile time.  For
// element offsets within a line, padx(j + r Q) = padx(j) + r Q + (r Q) / 32 when
// j < Q (Q a power of two: the low five bits of j + r Q do not carry), and
// likewise padx(e0 + r Ns) = padx(e0) + r Ns + (r Ns) / 32 for the stores
// (e0 = (j / Ns) Ns R + k with k < Ns), so every access of a butterfly is one base
// address plus a constant offset.
template <typename T, int R, int NTHR, int BPT, int SIGN, int LOG2P, int LOG2NS>
__device__ __forceinline__ void stockham_stage_fixed(c2<T> *buf, int ld, int nlines,
                                                     const c2<T> *__restrict__ tw) {
    constexpr int LOG2R = (R == 2) ? 1 : (R == 4) ? 2 : 4;
    constexpr int LOG2Q = LOG2P - LOG2R;
    constexpr int Q = 1 << LOG2Q;
    constexpr int Ns = 1 << LOG2NS;
    constexpr int TWSHIFT = LOG2P - LOG2NS - LOG2R;
    const int nb = nlines * Q;
    c2<T> v[BPT][R];
    int obase[BPT];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int f = threadIdx.x + b * NTHR;
        obase[b] = -1;
        if (f < nb) {
            const int line = f >> LOG2Q;
            const int j = f & (Q - 1);
            const int k = j & (Ns - 1);
            const c2<T> *pj = buf + line * ld + padx(j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = pj[r * Q + ((r * Q) >> 5)];
            if constexpr (LOG2NS > 0) {
                const int kt = k << TWSHIFT;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    c2<T> w = tw[r * kt];
                    if constexpr (SIGN > 0) w.y = -w.y;
                    v[b][r] = cmul<T>(v[b][r], w);
                }
            }
            dftR<T, R, SIGN>(v[b]);
            obase[b] = line * ld + padx(((j >> LOG2NS) << (LOG2NS + LOG2R)) + k);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        if (obase[b] >= 0) {
            c2<T> *pe = buf + obase[b];
#pragma unroll
            for (int r = 0; r < R; ++r) pe[r * Ns + ((r * Ns) >> 5)] = v[b][r];
        }
    }
    __syncthreads();
}

// lds_fft_dir for ODD = 1 and log2P = LOG2P fixed at compile time: radix-16 stages,
// then radix 4 and 2, as there
template <typename T, int NTHR, int BPT, int SIGN, int LOG2P, int LOG2NS = 0>
__device__ __forceinline__ void lds_fft_fixed(c2<T> *buf, int ld, int nlines, const c2<T> *__restrict__ tw) {
    constexpr int BPT16 = BPT / 4 > 0 ? BPT / 4 : 1;
    if constexpr (LOG2P - LOG2NS >= 4) {
        stockham_stage_fixed<T, 16, NTHR, BPT16, SIGN, LOG2P, LOG2NS>(buf, ld, nlines, tw);
        lds_fft_fixed<T, NTHR, BPT, SIGN, LOG2P, LOG2NS + 4>(buf, ld, nlines, tw);
    } else if constexpr (LOG2P - LOG2NS >= 2) {
        stockham_stage_fixed<T, 4, NTHR, BPT, SIGN, LOG2P, LOG2NS>(buf, ld, nlines, tw);
        lds_fft_fixed<T, NTHR, BPT, SIGN, LOG2P, LOG2NS + 2>(buf, ld, nlines, tw);
    } else if constexpr (LOG2P - LOG2NS == 1) {
        stockham_stage_fixed<T, 2, NTHR, 2 * BPT, SIGN, LOG2P, LOG2NS>(buf, ld, nlines, tw);
    }
}

// Lines of 2^p points take compile-time stages for the lengths in FIXSET (bit p),
// other lengths the general ones.  Kernels compile 2^9 .. 2^13 (the padded images
// and planes of the workloads); the four-step column passes also the short
// sub-transforms.  Every length compiled adds code to the kernel, and lengths it
// never sees cost registers and instruction cache.
constexpr unsigned kFixLong = 0x3e00u;   // 2^9 .. 2^13
constexpr unsigned kFixAll = 0x3fc0u;    // 2^6 .. 2^13

template <typename T, int NTHR, int BPT, int SIGN, unsigned FIXSET, int LOG2P>
__device__ __forceinline__ bool lds_fft_try(c2<T> *buf, int ld, int nlines, int log2P,
                                            const c2<T> *__restrict__ tw) {
    if constexpr ((FIXSET >> LOG2P) & 1u) {
        if (log2P == LOG2P) {
            lds_fft_fixed<T, NTHR, BPT, SIGN, LOG2P>(buf, ld, nlines, tw);
            return true;
        }
    }
    return false;
}

template <typename T, int NTHR, int BPT, int ODD, int SIGN, unsigned FIXSET>
__device__ __forceinline__ void lds_fft_sel(c2<T> *buf, int ld, int nlines, int log2P,
                                            const c2<T> *__restrict__ tw) {
    if constexpr (ODD == 1 && FIXSET != 0u) {
        if (lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 6>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 7>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 8>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 9>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 10>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 11>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 12>(buf, ld, nlines, log2P, tw) ||
            lds_fft_try<T, NTHR, BPT, SIGN, FIXSET, 13>(buf, ld, nlines, log2P, tw))
            return;
    }
    lds_fft_dir<T, NTHR, BPT, ODD, SIGN>(buf, ld, nlines, log2P, tw);
}

template <typename T, int NTHR, int BPT, int ODD = 1, unsigned FIXSET = kFixLong>
__device__ __forceinline__ void lds_fft(c2<T> *buf, int ld, int nlines, int log2P, int sign,
                                        const c2<T> *__restrict__ tw) {
    if (sign < 0) lds_fft_sel<T, NTHR, BPT, ODD, -1, FIXSET>(buf, ld, nlines, log2P, tw);
    else lds_fft_sel<T, NTHR, BPT, ODD, +1, FIXSET>(buf, ld, nlines, log2P, tw);
}

// Element idx of a batch of lines of length L = ODD 2^log2P: line idx / L, element idx % L.
template <int ODD> __device__ __forceinline__ int line_of(int idx, int log2P) { return div_odd<ODD>(idx >> log2P); }
template <int ODD> __device__ __forceinline__ int elem_of(int idx, int line, int L) {
    return (ODD == 1) ? (idx & (L - 1)) : idx - line * L;
}

// Workgroups go to the 8 XCDs round robin (linear id mod 8) and each XCD has its
// own L2.  Column-strip kernels, whose neighbouring strips share cache lines,
// renumber their work so that each XCD walks one contiguous range of strips:
// work = (lin mod 8) (n / 8) + lin / 8 when 8 divides the workgroup count n
// (a permutation of 0 .. n - 1; the identity otherwise).
__device__ __forceinline__ unsigned xcd_contiguous(unsigned lin, unsigned n) {
    return (n & 7u) ? lin : (lin & 7u) * (n >> 3) + (lin >> 3);
}

// store(idx, load(idx)) for idx = threadIdx.x, threadIdx.x + NTHR, ... < n, with U
// loads issued before their values are stored, so that U global loads per
// thread are in flight instead of one.
template <int NTHR, int U = 8, class Load, class Store>
__device__ __forceinline__ void staged_copy(int n, Load load, Store store) {
    for (int base = threadIdx.x; base < n; base += NTHR * U) {
        decltype(load(0)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * NTHR;
            if (idx < n) v[u] = load(idx);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * NTHR;
            if (idx < n) store(idx, v[u]);
        }
    }
}

// Twiddle table of a transform: copied into LDS (at twl) when the launcher
// reserved room for it (TWL), read from global memory otherwise.  The copy is
// complete at the caller's next barrier.
template <typename T, int NTHR, bool TWL>
__device__ __forceinline__ const c2<T> *stage_twiddles(c2<T> *twl, const c2<T> *__restrict__ tw, int L) {
    if constexpr (TWL) {
        staged_copy<NTHR>(L, [&](int i) { return tw[i]; }, [&](int i, c2<T> v) { twl[i] = v; });
        return twl;
    } else {
        return tw;
    }
}

// Rows per workgroup of the row transforms: about 4096 elements per workgroup
// (every thread busy in the radix-16 stages),
// fewer when there are too few rows to give every CU several workgroups.
inline int rows_per_wg(int L, int64_t nrows, int n_cu) {
    int lpw = std::max(1, 4096 / L);
    while (lpw > 1 && nrows / lpw < 4 * (int64_t)std::max(n_cu, 1)) lpw >>= 1;
    return lpw;
}

// LDS budget of one workgroup (bytes; gfx950 has 160 KiB per CU).
constexpr int kLdsBytes = 163840;

// Kernels using more than the default dynamic-LDS limit must opt in once.
template <typename F>
inline void allow_lds(F *func, size_t bytes) {
    // the attribute is raised once per kernel and device to the largest size asked for
    if (bytes <= 65536) return;
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, size_t> done;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    size_t &have = done[{dev, (const void *)func}];
    if (have >= bytes) return;
    HIP_CHECK(hipFuncSetAttribute((const void *)func, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    have = bytes;
}

}  // namespace frmi
