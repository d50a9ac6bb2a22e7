// Shared device/host helpers of the HIP library: complex type, fast unsigned
// division by a run-time constant, status plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qf.h"

namespace qf {

// Interleaved complex number with the memory layout of torch.complex64/128.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cplx<T> cmake(T r, T i) {
    cplx<T> c;
    c.re = r;
    c.im = i;
    return c;
}

template <typename T>
__host__ __device__ inline cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return cmake<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}

template <typename T>
__host__ __device__ inline cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return cmake<T>(a.re + b.re, a.im + b.im);
}

template <typename T>
__host__ __device__ inline cplx<T> cconj(cplx<T> a) {
    return cmake<T>(a.re, -a.im);
}

// acc += a * b
template <typename T>
__host__ __device__ inline void cmac(cplx<T>& acc, cplx<T> a, cplx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}

// acc += conj(a) * b
template <typename T>
__host__ __device__ inline void cmac_conj(cplx<T>& acc, cplx<T> a, cplx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}

// Division of 32-bit unsigned numerators by a fixed divisor d >= 1 with one
// multiply-high, an add and a shift (Granlund & Montgomery, "Division by
// invariant integers using multiplication", PLDI 1994: the round-up multiplier
// m = ceil(2^(32+s) / d), s = ceil(log2 d), stored as m - 2^32).
struct FastDiv {
    uint32_t d;
    uint32_t mprime;
    uint32_t s;

    __host__ __device__ FastDiv() : d(1), mprime(0), s(0) {}
    __host__ explicit FastDiv(uint32_t div) { init(div); }

    __host__ void init(uint32_t div) {
        d = div;
        s = 0;
        while ((uint64_t(1) << s) < uint64_t(div)) ++s;
        // s reaches 32 for divisors above 2^31 (registers of more than 2^31
        // amplitudes), so 2^(32+s) needs 128-bit arithmetic; m - 2^32 still
        // fits in 32 bits because 2^(32+s) / d < 2^33.
        const unsigned __int128 one = 1;
        const unsigned __int128 m = ((one << (32 + s)) + div - 1) / div;
        mprime = uint32_t(uint64_t(m - (one << 32)));
    }

    __device__ inline uint32_t div(uint32_t n) const {
        uint64_t t = uint64_t(__umulhi(n, mprime)) + n;
        return uint32_t(t >> s);
    }
    __host__ inline uint32_t div_host(uint32_t n) const {
        uint64_t hi = (uint64_t(n) * mprime) >> 32;
        return uint32_t((hi + n) >> s);
    }
};

}  // namespace qf

// ---------------------------------------------------------------------------
// Host-side status helpers (defined in abi.cpp).
// ---------------------------------------------------------------------------
namespace qf {
qf_status set_error(qf_status st, const char* fmt, ...);
qf_status check_launch(const char* what);
// Every device and pinned-host allocation of the library goes through these.
// With the environment variable QF_TEST_FAIL_ALLOC set to a non-zero value they
// fail with QF_ENOMEM before calling HIP (failure injection for tests).
qf_status dev_malloc(void** p, size_t bytes, const char* what);
qf_status dev_malloc_async(void** p, size_t bytes, hipStream_t st, const char* what);
// Returns the freed memory the default pools keep (every device the library used).
void trim_pools();
qf_status host_malloc_pinned(void** p, size_t bytes, const char* what);
// QF_LOG set to a non-zero value: planner and autotuner choices go to stderr.
bool log_enabled();
void log_msg(const char* fmt, ...);
}  // namespace qf

#define QF_RETURN_IF(cond, st, ...)                      \
    do {                                                 \
        if (cond) return ::qf::set_error((st), __VA_ARGS__); \
    } while (0)

#define QF_HIP_CHECK(call)                                                        \
    do {                                                                          \
        hipError_t _e = (call);                                                   \
        if (_e != hipSuccess)                                                     \
            return ::qf::set_error(QF_EHIP, "%s failed: %s", #call, hipGetErrorString(_e)); \
    } while (0)

#define QF_CHECK(call)                 \
    do {                               \
        qf_status _s = (call);         \
        if (_s != QF_OK) return _s;    \
    } while (0)
