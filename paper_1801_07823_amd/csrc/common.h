// Shared device/host helpers for the KD-MG library: complex arithmetic on
// plain structs (FP64, FP32 and FP16 storage), launch checks, and the status
// plumbing of the C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <stdexcept>
#include <string>

#include "../../include/kdmg.h"

namespace kdmg {

// --------------------------------------------------------------- complex

template <class R>
struct alignas(2 * sizeof(R)) Cx {
  R re, im;
};

using c64 = Cx<double>;
using c32 = Cx<float>;
using c16 = Cx<_Float16>;

template <class R>
__host__ __device__ __forceinline__ Cx<R> mk(R a, R b) { return Cx<R>{a, b}; }

// widen/narrow a storage value to the compute type
template <class R, class S>
__host__ __device__ __forceinline__ Cx<R> ld(const Cx<S>& s) {
  return Cx<R>{(R)s.re, (R)s.im};
}
template <class S, class R>
__host__ __device__ __forceinline__ Cx<S> st(const Cx<R>& v) {
  return Cx<S>{(S)v.re, (S)v.im};
}

template <class R>
__host__ __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator-(Cx<R> a) { return {-a.re, -a.im}; }
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.re, s * a.im}; }
template <class R>
__host__ __device__ __forceinline__ Cx<R>& operator+=(Cx<R>& a, Cx<R> b) { a.re += b.re; a.im += b.im; return a; }
template <class R>
__host__ __device__ __forceinline__ Cx<R>& operator-=(Cx<R>& a, Cx<R> b) { a.re -= b.re; a.im -= b.im; return a; }
template <class R>
__host__ __device__ __forceinline__ Cx<R> conj(Cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class R>
__host__ __device__ __forceinline__ Cx<R> cmul_conj(Cx<R> a, Cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc += a * b
template <class R>
__host__ __device__ __forceinline__ void cfma(Cx<R>& acc, Cx<R> a, Cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <class R>
__host__ __device__ __forceinline__ void cfma_conj(Cx<R>& acc, Cx<R> a, Cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
template <class R>
__host__ __device__ __forceinline__ R norm2(Cx<R> a) { return a.re * a.re + a.im * a.im; }

// --------------------------------------------------------------- errors

struct Error : std::runtime_error {
  kdmg_status code;
  Error(kdmg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define KDMG_HIP(call)                                                           \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::kdmg::Error(KDMG_EHIP, std::string(#call " failed: ") +            \
                                         hipGetErrorString(e_) + " at " +        \
                                         __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

#define KDMG_CHECK(cond, code, msg)                                              \
  do {                                                                           \
    if (!(cond)) throw ::kdmg::Error((code), (msg));                             \
  } while (0)

#define KDMG_LAUNCH_CHECK() KDMG_HIP(hipGetLastError())

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// --------------------------------------------------------------- device memory

// Serialises the library's device and pinned allocations and frees with its
// hipGraph captures: a free synchronises the device, which must not happen
// while another thread has a stream in capture.
inline std::mutex& hip_mem_mutex() {
  static std::mutex m;
  return m;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    std::lock_guard<std::mutex> g(hip_mem_mutex());
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(KDMG_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
  }
  void release() {
    if (p) {
      std::lock_guard<std::mutex> g(hip_mem_mutex());
      (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace kdmg
