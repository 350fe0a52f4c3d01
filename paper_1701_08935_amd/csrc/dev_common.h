// Device-side scalar types and helpers (gfx950, HIP).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace zolo {

struct zd {
  double re, im;
};
struct zf {
  float re, im;
};

// ---- global-memory access ---------------------------------------------------
// Pointers read from descriptor arrays are generic (flat) pointers.  Accessing
// them through the global address space lets the compiler emit global loads
// and stores, whose completion counter is separate from the LDS one; a flat
// load would make every later LDS wait also wait for it.
typedef __attribute__((address_space(1))) const double* gcdp;
typedef __attribute__((address_space(1))) double* gdp;
typedef __attribute__((address_space(1))) const float* gcfp;
typedef __attribute__((address_space(1))) float* gfp;
__device__ inline double gld(const double* p) { return *(gcdp)p; }
__device__ inline float gld(const float* p) { return *(gcfp)p; }
__device__ inline void gst(double* p, double v) { *(gdp)p = v; }
__device__ inline void gst(float* p, float v) { *(gfp)p = v; }
typedef double dpair __attribute__((ext_vector_type(2)));
typedef float fpair __attribute__((ext_vector_type(2)));
__device__ inline zd gld(const zd* p) {
  dpair v = *(__attribute__((address_space(1))) const dpair*)p;
  return zd{v.x, v.y};
}
__device__ inline zf gld(const zf* p) {
  fpair v = *(__attribute__((address_space(1))) const fpair*)p;
  return zf{v.x, v.y};
}
__device__ inline void gst(zd* p, const zd& v) { *(__attribute__((address_space(1))) dpair*)p = dpair{v.re, v.im}; }
__device__ inline void gst(zf* p, const zf& v) { *(__attribute__((address_space(1))) fpair*)p = fpair{v.re, v.im}; }

// ---- scalar traits --------------------------------------------------------
template <typename T>
struct ST;

template <>
struct ST<double> {
  typedef double real;
  static constexpr bool cplx = false;
  __host__ __device__ static inline double zero() { return 0.0; }
  __host__ __device__ static inline double one() { return 1.0; }
};
template <>
struct ST<float> {
  typedef float real;
  static constexpr bool cplx = false;
  __host__ __device__ static inline float zero() { return 0.0f; }
  __host__ __device__ static inline float one() { return 1.0f; }
};
template <>
struct ST<zd> {
  typedef double real;
  static constexpr bool cplx = true;
  __host__ __device__ static inline zd zero() { return zd{0.0, 0.0}; }
  __host__ __device__ static inline zd one() { return zd{1.0, 0.0}; }
};
template <>
struct ST<zf> {
  typedef float real;
  static constexpr bool cplx = true;
  __host__ __device__ static inline zf zero() { return zf{0.0f, 0.0f}; }
  __host__ __device__ static inline zf one() { return zf{1.0f, 0.0f}; }
};

// ---- arithmetic -----------------------------------------------------------
__host__ __device__ inline double mul(double a, double b) { return a * b; }
__host__ __device__ inline float mul(float a, float b) { return a * b; }
__host__ __device__ inline zd mul(zd a, zd b) { return zd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline zf mul(zf a, zf b) { return zf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__host__ __device__ inline double add(double a, double b) { return a + b; }
__host__ __device__ inline float add(float a, float b) { return a + b; }
__host__ __device__ inline zd add(zd a, zd b) { return zd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline zf add(zf a, zf b) { return zf{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline double sub(double a, double b) { return a - b; }
__host__ __device__ inline float sub(float a, float b) { return a - b; }
__host__ __device__ inline zd sub(zd a, zd b) { return zd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline zf sub(zf a, zf b) { return zf{a.re - b.re, a.im - b.im}; }
// a + b*c
__host__ __device__ inline double fma_(double a, double b, double c) { return fma(b, c, a); }
__host__ __device__ inline float fma_(float a, float b, float c) { return fmaf(b, c, a); }
__host__ __device__ inline zd fma_(zd a, zd b, zd c) {
  return zd{fma(b.re, c.re, fma(-b.im, c.im, a.re)), fma(b.re, c.im, fma(b.im, c.re, a.im))};
}
__host__ __device__ inline zf fma_(zf a, zf b, zf c) {
  return zf{fmaf(b.re, c.re, fmaf(-b.im, c.im, a.re)), fmaf(b.re, c.im, fmaf(b.im, c.re, a.im))};
}
__host__ __device__ inline double conj_(double a) { return a; }
__host__ __device__ inline float conj_(float a) { return a; }
__host__ __device__ inline zd conj_(zd a) { return zd{a.re, -a.im}; }
__host__ __device__ inline zf conj_(zf a) { return zf{a.re, -a.im}; }
__host__ __device__ inline double inv_(double a) { return 1.0 / a; }
__host__ __device__ inline float inv_(float a) { return 1.0f / a; }
__host__ __device__ inline zd inv_(zd a) {
  // Smith's algorithm for 1 / (re + i im)
  if (fabs(a.re) >= fabs(a.im)) {
    double r = a.im / a.re, d = a.re + a.im * r;
    return zd{1.0 / d, -r / d};
  } else {
    double r = a.re / a.im, d = a.re * r + a.im;
    return zd{r / d, -1.0 / d};
  }
}
__host__ __device__ inline zf inv_(zf a) {
  if (fabsf(a.re) >= fabsf(a.im)) {
    float r = a.im / a.re, d = a.re + a.im * r;
    return zf{1.0f / d, -r / d};
  } else {
    float r = a.re / a.im, d = a.re * r + a.im;
    return zf{r / d, -1.0f / d};
  }
}
__host__ __device__ inline double neg(double a) { return -a; }
__host__ __device__ inline float neg(float a) { return -a; }
__host__ __device__ inline zd neg(zd a) { return zd{-a.re, -a.im}; }
__host__ __device__ inline zf neg(zf a) { return zf{-a.re, -a.im}; }
__host__ __device__ inline double abs2(double a) { return a * a; }
__host__ __device__ inline float abs2(float a) { return a * a; }
__host__ __device__ inline double abs2(zd a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline float abs2(zf a) { return a.re * a.re + a.im * a.im; }

__host__ __device__ inline double re_(double a) { return a; }
__host__ __device__ inline double re_(zd a) { return a.re; }
__host__ __device__ inline double scl(double a, double r) { return a * r; }
__host__ __device__ inline zd scl(zd a, double r) { return zd{a.re * r, a.im * r}; }

// conversions
template <typename To, typename From>
__host__ __device__ inline To cvt(From x);
template <>
__host__ __device__ inline double cvt<double, double>(double x) { return x; }
template <>
__host__ __device__ inline zd cvt<zd, double>(double x) { return zd{x, 0.0}; }
template <>
__host__ __device__ inline zf cvt<zf, double>(double x) { return zf{(float)x, 0.0f}; }
template <>
__host__ __device__ inline zd cvt<zd, zd>(zd x) { return x; }
template <>
__host__ __device__ inline zf cvt<zf, zd>(zd x) { return zf{(float)x.re, (float)x.im}; }
template <>
__host__ __device__ inline zd cvt<zd, zf>(zf x) { return zd{(double)x.re, (double)x.im}; }
template <>
__host__ __device__ inline zf cvt<zf, zf>(zf x) { return x; }
template <>
__host__ __device__ inline float cvt<float, double>(double x) { return (float)x; }
template <>
__host__ __device__ inline double cvt<double, float>(float x) { return (double)x; }
// real factorizations (real shifts of real pencils, for inertia counts) take the
// real part of an entry whose imaginary part is zero by construction
template <>
__host__ __device__ inline double cvt<double, zd>(zd x) { return x.re; }

}  // namespace zolo
