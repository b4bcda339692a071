// Internal definitions shared by the HIP translation units of libfrmi.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/frmi.h"

namespace frmi {

// ----------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string &m);

#define FR_REQUIRE(cond, msg)                                                        \
    do {                                                                             \
        if (!(cond)) throw ::frmi::Error(FR_EINVAL, std::string(__func__) + ": " + (msg)); \
    } while (0)

#define HIP_CHECK(expr)                                                              \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            int code_ = (e_ == hipErrorOutOfMemory) ? FR_ENOMEM : FR_EHIP;          \
            throw ::frmi::Error(code_, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                            \
    } while (0)

#define LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

// ----------------------------------------------------------------- complex
template <typename T> struct C2T;
template <> struct C2T<float> { using type = float2; };
template <> struct C2T<double> { using type = double2; };
template <typename T> using c2 = typename C2T<T>::type;

template <typename T> __host__ __device__ __forceinline__ c2<T> mk(T x, T y) {
    c2<T> r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename T> __device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ c2<T> cconj(c2<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ c2<T> cscale(c2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// sin/cos of 2 pi x for x in cycles (x reduced by the caller to about [-1, 1]).
__device__ __forceinline__ void sincos_cycles(float x, float *s, float *c) { sincospif(2.0f * x, s, c); }
__device__ __forceinline__ void sincos_cycles(double x, double *s, double *c) { sincospi(2.0 * x, s, c); }

// ----------------------------------------------------------------- context
constexpr int kMaxLog2FFT = 14;  // FFT lengths 2 .. 16384
constexpr int kMaxLog2Odd = 13;  // tables of lengths 3 2^p and 5 2^p, p <= 13

struct Ctx {
    void *owner = nullptr;  // the fr_ctx holding this context
    int device = 0;
    int n_cu = 0;
    // twiddle tables tw[m] = exp(-2 pi i m / L), m < L, per log2 L, per precision;
    // tw*o[0] for L = 3 2^p, tw*o[1] for L = 5 2^p
    void *tw32[kMaxLog2FFT + 2] = {};
    void *tw64[kMaxLog2FFT + 2] = {};
    void *tw32o[2][kMaxLog2Odd + 1] = {};
    void *tw64o[2][kMaxLog2Odd + 1] = {};
    template <typename T> const c2<T> *tw(int log2L) const;
    // table of L = odd 2^log2P, odd in {1, 3, 5}
    template <typename T> const c2<T> *tw(int odd, int log2P) const {
        if (odd == 1) return tw<T>(log2P);
        void *const(*t)[kMaxLog2Odd + 1] = sizeof(T) == 8 ? tw64o : tw32o;
        return (const c2<T> *)t[odd == 3 ? 0 : 1][log2P];
    }
};
template <> inline const float2 *Ctx::tw<float>(int l) const { return (const float2 *)tw32[l]; }
template <> inline const double2 *Ctx::tw<double>(int l) const { return (const double2 *)tw64[l]; }

inline int ilog2(int64_t n) {
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}
inline bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// Host side: n = odd 2^log2P with odd in {1, 3, 5}; false for other lengths.
inline bool split_len(int64_t n, int *odd, int *log2P) {
    if (n <= 0) return false;
    int o = 1;
    if (n % 3 == 0) o = 3;
    else if (n % 5 == 0) o = 5;
    const int64_t p = n / o;
    if (p & (p - 1)) return false;
    int l = 0;
    while ((int64_t(1) << l) < p) ++l;
    *odd = o;
    *log2P = l;
    return true;
}

// f(std::integral_constant<int, ODD>{}) for a runtime odd factor in {1, 3, 5}
template <class F> inline void with_odd(int odd, F &&f) {
    switch (odd) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        default: throw Error(FR_EINVAL, "line lengths must be 2^p, 3 2^p or 5 2^p");
    }
}

// Device allocations of the library (hipMalloc).  A test hook can make the
// allocation after the next `n` succeed fail as if the device were out of memory
// (fr_inject_alloc_failure), to exercise the error paths.
hipError_t device_alloc(void **p, size_t bytes);

// Bytes a Scratch of `bytes` takes from its arena (regions are 256-byte aligned).
constexpr size_t scratch_round(size_t bytes) { return (bytes + 255) & ~size_t(255); }

// Scratch memory of library calls on one stream, kept from call to call: a stack
// of device chunks that only grows (a chunk is added when a request does not fit;
// the first calls on a stream pay for it).  Work on a stream runs in order, so a
// region released at the end of one call is free for the next call on the same
// stream, and no allocation or release is enqueued per call (a stream-ordered
// allocate/free pair costs 10-20 us of stream time on this runtime).  Regions are
// released in reverse order of acquisition (RAII scopes).  Each (device, stream)
// has its own arena; its memory is held until the process ends.
class Arena {
  public:
    struct Mark {
        int chunk = 0;
        size_t top = 0;
        size_t live = 0;
    };
    void *push(size_t bytes, Mark &m) {
        std::lock_guard<std::mutex> g(mu_);
        const size_t b = scratch_round(bytes);
        if (chunks_.empty()) add_chunk(std::max<size_t>(b, size_t(64) << 20));
        // on failure below nothing has moved: the caller's regions stay as they were
        int cur = cur_;
        size_t top = top_;
        while (top + b > chunks_[cur].cap) {
            if (cur + 1 == (int)chunks_.size()) add_chunk(std::max(b, 2 * chunks_[cur].cap));
            ++cur;
            top = 0;
        }
        m.chunk = cur_;
        m.top = top_;
        m.live = live_;
        cur_ = cur;
        void *p = chunks_[cur].p + top;
        top_ = top + b;
        live_ += b;
        peak_ = std::max(peak_, live_);
        return p;
    }
    void pop(const Mark &m) {
        std::lock_guard<std::mutex> g(mu_);
        cur_ = m.chunk;
        top_ = m.top;
        live_ = m.live;
    }
    size_t held() {
        std::lock_guard<std::mutex> g(mu_);
        size_t t = 0;
        for (auto &c : chunks_) t += c.cap;
        return t;
    }
    // highest sum of live region sizes since the last reset
    size_t peak(bool reset) {
        std::lock_guard<std::mutex> g(mu_);
        const size_t v = peak_;
        if (reset) peak_ = live_;
        return v;
    }
    // Free every chunk; false (nothing freed) while a region is live.  The caller
    // has synchronised the stream, so no enqueued work still uses the memory.
    bool trim() {
        std::lock_guard<std::mutex> g(mu_);
        if (live_ != 0) return false;
        for (auto &c : chunks_) (void)hipFree(c.p);
        chunks_.clear();
        cur_ = 0;
        top_ = 0;
        return true;
    }

  private:
    struct Chunk {
        char *p;
        size_t cap;
    };
    void add_chunk(size_t cap) {
        void *p = nullptr;
        const hipError_t e = device_alloc(&p, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(FR_ENOMEM, "scratch allocation of " + std::to_string(cap) + " bytes failed");
        }
        chunks_.push_back({(char *)p, cap});
    }
    std::mutex mu_;
    std::vector<Chunk> chunks_;
    int cur_ = 0;
    size_t top_ = 0;
    size_t live_ = 0, peak_ = 0;
};

// the arena of (current device, stream)
Arena &arena_for(hipStream_t st);

struct Scratch {
    void *p = nullptr;
    Arena *a = nullptr;
    Arena::Mark m;
    Scratch() = default;
    Scratch(size_t bytes, hipStream_t st) {
        if (bytes) {
            a = &arena_for(st);
            p = a->push(bytes, m);
        }
    }
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    Scratch(Scratch &&o) noexcept : p(o.p), a(o.a), m(o.m) { o.p = nullptr; }
    Scratch &operator=(Scratch &&o) noexcept {
        if (this != &o) {
            if (p) a->pop(m);
            p = o.p;
            a = o.a;
            m = o.m;
            o.p = nullptr;
        }
        return *this;
    }
    ~Scratch() {
        if (p) a->pop(m);
    }
    template <typename U> U *as() const { return (U *)p; }
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) HIP_CHECK(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
    }
};

// owning device buffer
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) : bytes(n) {
        if (n) HIP_CHECK(device_alloc(&p, n));
    }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            if (p) (void)hipFree(p);
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    template <typename U> U *as() const { return (U *)p; }
};

}  // namespace frmi
