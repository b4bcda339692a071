// Generic complex-to-complex line-FFT kernels with load/store functors.
//
//   k_fft_rows: each workgroup transforms `lines_per_wg` rows; element e of row r
//               is read with pro(r, e) and written with epi(r, e, value).
//   k_fft_cols: each workgroup transforms a strip of C adjacent columns of one
//               [rows][cols] matrix (strips of all matrices in XCD-contiguous order); only the first
//               n_in rows are read (the rest are known zeros) and the first n_out
//               rows are written.  Row-segment reads of C consecutive elements keep
//               the global accesses coalesced; columns are transposed into padded
//               LDS lines (stride L + 1) on the way in and out.
#pragma once

#include "fft.h"

namespace frmi {

template <typename T, int NTHR, int BPT, bool TWL, class Pro, class Epi, int ODD = 1>
__global__ __launch_bounds__(NTHR) void k_fft_rows(Pro pro, Epi epi, int64_t nrows, int log2P,
                                                    int lines_per_wg, int sign,
                                                    const c2<T> *__restrict__ tw) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int L = ODD << log2P;
    const int64_t row0 = (int64_t)blockIdx.x * lines_per_wg;
    const int nl = (int)min<int64_t>(lines_per_wg, nrows - row0);
    const int ld = plen(L);
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + lines_per_wg * ld, tw, L);
    staged_copy<NTHR>(
        nl * L,
        [&](int idx) {
            const int c = line_of<ODD>(idx, log2P);
            return pro(row0 + c, elem_of<ODD>(idx, c, L));
        },
        [&](int idx, c2<T> v) {
            const int c = line_of<ODD>(idx, log2P);
            buf[c * ld + padx(elem_of<ODD>(idx, c, L))] = v;
        });
    __syncthreads();
    lds_fft<T, NTHR, BPT, ODD>(buf, ld, nl, log2P, sign, twp);
    for (int idx = threadIdx.x; idx < nl * L; idx += NTHR) {
        const int c = line_of<ODD>(idx, log2P), e = elem_of<ODD>(idx, c, L);
        epi(row0 + c, e, buf[c * ld + padx(e)]);
    }
}

template <typename T, int NTHR, int BPT, bool TWL, class Pro, class Epi, int ODD = 1>
__global__ __launch_bounds__(NTHR) void k_fft_cols(Pro pro, Epi epi, int ncols, int log2P, int n_in,
                                                    int n_out, int C, int sign,
                                                    const c2<T> *__restrict__ tw,
                                                    const int32_t *__restrict__ blk, int log2_spb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    c2<T> *buf = reinterpret_cast<c2<T> *>(smem_raw);
    const int L = ODD << log2P;
    const int ld = plen(L) + 1;
    const unsigned w = xcd_contiguous(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const unsigned s = w % gridDim.x;
    const int64_t m = w / gridDim.x;
    const int log2C = 31 - __builtin_clz(C);  // strips are a power of two wide
    // strip s: with a block list, strip s & (2^log2_spb - 1) of column block
    // blk[s >> log2_spb] (blocks of C 2^log2_spb columns); else columns s C ..
    const int col0 = blk ? (blk[s >> log2_spb] << (log2_spb + log2C)) + (int)((s & ((1u << log2_spb) - 1u)) << log2C)
                         : (int)s * C;
    const c2<T> *twp = stage_twiddles<T, NTHR, TWL>(buf + C * ld, tw, L);
    staged_copy<NTHR>(
        C * L,
        [&](int idx) {
            const int r = idx >> log2C, c = idx & (C - 1);
            return (r < n_in) ? pro(m, r, col0 + c) : mk<T>(T(0), T(0));
        },
        [&](int idx, c2<T> v) {
            const int r = idx >> log2C, c = idx & (C - 1);
            buf[c * ld + padx(r)] = v;
        });
    __syncthreads();
    lds_fft<T, NTHR, BPT, ODD>(buf, ld, C, log2P, sign, twp);
    for (int idx = threadIdx.x; idx < C * n_out; idx += NTHR) {
        const int r = idx >> log2C, c = idx & (C - 1);
        epi(m, r, col0 + c, buf[c * ld + padx(r)]);
    }
}

// dynamic LDS of a line transform: the lines, plus the twiddle table when it fits
template <typename T> inline bool twl_fits(size_t data_bytes, int L) {
    return data_bytes + (size_t)L * sizeof(c2<T>) <= (size_t)kLdsBytes;
}

// Row transforms of length L = ODD 2^log2P.
template <typename T, class Pro, class Epi, int ODD = 1>
void launch_fft_rows(const Ctx &ctx, Pro pro, Epi epi, int64_t nrows, int log2P, int sign, hipStream_t st) {
    const int L = ODD << log2P;
    FR_REQUIRE((int64_t)plen(L) * (int64_t)sizeof(c2<T>) <= kLdsBytes && L <= 16384, "FFT length too large");
    if (nrows <= 0) return;
    const c2<T> *tw = ctx.tw<T>(ODD, log2P);
    const size_t pline = (size_t)plen(L) * sizeof(c2<T>);
    if (L <= 4096) {
        const int lpw = rows_per_wg(L, nrows, ctx.n_cu);
        const size_t lds = (size_t)lpw * pline + (size_t)L * sizeof(c2<T>);
        allow_lds(k_fft_rows<T, 256, 4, true, Pro, Epi, ODD>, lds);
        k_fft_rows<T, 256, 4, true, Pro, Epi, ODD><<<dim3((unsigned)((nrows + lpw - 1) / lpw)), 256, lds, st>>>(
            pro, epi, nrows, log2P, lpw, sign, tw);
    } else if (L < 8192 && twl_fits<T>(pline, L)) {
        const size_t lds = pline + (size_t)L * sizeof(c2<T>);
        allow_lds(k_fft_rows<T, 512, 4, true, Pro, Epi, ODD>, lds);
        k_fft_rows<T, 512, 4, true, Pro, Epi, ODD><<<dim3((unsigned)nrows), 512, lds, st>>>(pro, epi, nrows, log2P,
                                                                                         1, sign, tw);
    } else {
        // lines of 8192 and more: no LDS twiddle table, so that two workgroups fit
        // per CU (8192^2 planes: 33% faster than one workgroup with the table)
        const size_t lds = pline;
        allow_lds(k_fft_rows<T, 1024, 4, false, Pro, Epi, ODD>, lds);
        k_fft_rows<T, 1024, 4, false, Pro, Epi, ODD><<<dim3((unsigned)nrows), 1024, lds, st>>>(pro, epi, nrows,
                                                                                            log2P, 1, sign, tw);
    }
    LAUNCH_CHECK();
}

// Column strip width: as many columns as keep the LDS lines within 64 KiB (two
// workgroups per CU), at most 16, a divisor of ncols.
template <typename T> inline int col_strip(int L, int ncols) {
    const int cap = std::max(1, std::min(16, (int)(65536 / sizeof(c2<T>)) / L));
    int C = 1;
    while (2 * C <= cap) C *= 2;
    while (C > 1 && (ncols % C)) C >>= 1;
    return C;
}

// Column transforms of length L = ODD 2^log2P, of every column, or with blk (device
// int32 [nblk]) only of the columns of blocks blk[0 .. nblk - 1], each blk_w (a
// power of two) columns wide.
template <typename T, class Pro, class Epi, int ODD = 1>
void launch_fft_cols(const Ctx &ctx, Pro pro, Epi epi, int64_t nmat, int ncols, int log2P, int n_in, int n_out,
                     int sign, hipStream_t st, const int32_t *blk = nullptr, int nblk = 0, int blk_w = 0) {
    const int L = ODD << log2P;
    if (blk) {
        FR_REQUIRE(is_pow2(blk_w) && blk_w <= ncols, "column blocks must be a power of two wide");
        ncols = nblk * blk_w;  // the columns transformed
    }
    int C = col_strip<T>(L, ncols);
    bool allow_twl = true;
    // FP32 lines of 8192: strips of two columns without the LDS twiddle table
    // (twiddles then come through the caches) move 16 bytes per row access instead
    // of 8; measured 20% faster than one column with the table on 8192^2 planes
    if (sizeof(T) == 4 && L == 8192 && ncols % 2 == 0) {
        C = 2;
        allow_twl = false;
    }
    // few matrices (e.g. three Taylor planes): narrower strips so the grid still
    // covers every CU a couple of times
    while (C > 2 && (int64_t)(ncols / C) * nmat < 2 * (int64_t)std::max(ctx.n_cu, 1)) C >>= 1;
    FR_REQUIRE(is_pow2(C), "column strip width must be a power of two");
    if (blk) C = std::min(C, blk_w);
    const int log2_spb = blk ? ilog2(blk_w / C) : 0;
    const size_t lds = (size_t)C * (plen(L) + 1) * sizeof(c2<T>);
    FR_REQUIRE(lds <= (size_t)kLdsBytes && L <= 16384, "column FFT length too large");
    if (nmat <= 0 || ncols <= 0) return;
    dim3 grid((unsigned)(ncols / C), (unsigned)nmat);
    const bool twl = allow_twl && twl_fits<T>(lds, L);
    const size_t ldst = twl ? lds + (size_t)L * sizeof(c2<T>) : lds;
#define FR_COLS(NT, TW)                                                                                   \
    do {                                                                                                  \
        allow_lds(k_fft_cols<T, NT, 4, TW, Pro, Epi, ODD>, ldst);                                              \
        k_fft_cols<T, NT, 4, TW, Pro, Epi, ODD><<<grid, NT, ldst, st>>>(pro, epi, ncols, log2P, n_in, n_out, C, \
                                                                   sign, ctx.tw<T>(ODD, log2P), blk, log2_spb); \
    } while (0)
    // one radix-4 butterfly per thread where the strip allows (as the convolution
    // column pass)
    if (C * L <= 1024) {
        if (twl) FR_COLS(256, true);
        else FR_COLS(256, false);
    } else if (C * L <= 2048) {
        if (twl) FR_COLS(512, true);
        else FR_COLS(512, false);
    } else {
        if (twl) FR_COLS(1024, true);
        else FR_COLS(1024, false);
    }
#undef FR_COLS
    LAUNCH_CHECK();
}

// plain strided complex matrix access: base + m * mstride + r * ncols + c
template <typename T> struct MatLoad {
    const c2<T> *base;
    int64_t mstride;
    int ncols;
    __device__ c2<T> operator()(int64_t m, int r, int c) const { return base[m * mstride + (int64_t)r * ncols + c]; }
};
template <typename T> struct MatStore {
    c2<T> *base;
    int64_t mstride;
    int ncols;
    __device__ void operator()(int64_t m, int r, int c, c2<T> v) const { base[m * mstride + (int64_t)r * ncols + c] = v; }
};
template <typename T> struct RowLoad {
    const c2<T> *base;
    int64_t L;
    __device__ c2<T> operator()(int64_t r, int e) const { return base[r * L + e]; }
};
template <typename T> struct RowStore {
    c2<T> *base;
    int64_t L;
    __device__ void operator()(int64_t r, int e, c2<T> v) const { base[r * L + e] = v; }
};

}  // namespace frmi
