// Shared definitions of the gfx950 integral-equation library: complex arithmetic, error
// reporting, launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "ie.h"

namespace ie {

// ---------------------------------------------------------------------------------------
// complex numbers (interleaved re, im), T = double (complex128) or float (complex64)
// ---------------------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// a + b * c
template <typename T>
__host__ __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re};
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cx<To> ccast(cx<Ti> a) { return {To(a.re), To(a.im)}; }

using c64 = cx<float>;
using c128 = cx<double>;

// ---------------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);  // records the message, returns code

#define IE_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::ie::fail(IE_EDEVICE, "%s failed at %s:%d: %s", #call, __FILE__, __LINE__, \
                        hipGetErrorString(e_));                                          \
  } while (0)

#define IE_TRY(call)          \
  do {                        \
    int s_ = (call);          \
    if (s_ < 0) return s_;    \
  } while (0)

#define IE_LAUNCH_CHECK() IE_HIP(hipGetLastError())

inline int ceil_div(long a, long b) { return int((a + b - 1) / b); }

// FFT twiddle table length: entries exp(-2 pi i k / TW_N); every FFT length (2^k or 3 * 2^k up
// to MAX_FFT_LEN) divides TW_N and reads its twiddles at stride TW_N / L.
constexpr int TW_N = 3072;
constexpr int MAX_FFT_LEN = 1024;

// A field view: element (c, z, y, x) at p[c * cs + ((z - zoff) * ny + y) * nx + x].
template <typename T>
struct View {
  T* p;
  long cs;
  int zoff;
};

}  // namespace ie
