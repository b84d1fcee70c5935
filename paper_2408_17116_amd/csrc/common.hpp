// Shared device/host helpers of the CBIE H-matrix library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace cbie {

// ---------------------------------------------------------------- complex
template <typename T> struct cplx { T re, im; };
using zd = cplx<double>;
using zf = cplx<float>;

template <typename T> __host__ __device__ inline cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T> __host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a) { return {-a.re, -a.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ inline T abs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ inline cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    // Smith's algorithm: avoids overflow of |b|^2
    if (fabs(b.re) >= fabs(b.im)) {
        T r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        T r = b.re / b.im, d = b.re * r + b.im;
        return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}
// a += b * c
template <typename T> __host__ __device__ inline void cfma(cplx<T>& a, cplx<T> b, cplx<T> c) {
    a.re = fma(b.re, c.re, a.re); a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im); a.im = fma(b.im, c.re, a.im);
}

// ----------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};

#define CBIE_HIP(call)                                                              \
    do {                                                                            \
        hipError_t _e = (call);                                                     \
        if (_e != hipSuccess)                                                       \
            throw ::cbie::Error{-3, std::string(#call) + ": " + hipGetErrorString(_e)}; \
    } while (0)

#define CBIE_REQUIRE(cond, code, text)                                              \
    do {                                                                            \
        if (!(cond)) throw ::cbie::Error{(code), std::string(text)};               \
    } while (0)

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string(what) + ": " + hipGetErrorString(e)};
}

// ------------------------------------------------------- device buffers
template <typename T> struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr; n = 0;
    }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{-2, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
        }
        n = count;
    }
    void upload(const T* h, size_t count, hipStream_t s) {
        if (count > n) alloc(count);
        if (count) CBIE_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
    void download(T* h, size_t count, hipStream_t s) const {
        if (count) CBIE_HIP(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
    }
};

inline unsigned ceil_div(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace cbie
