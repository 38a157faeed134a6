// Shared device/host helpers of the gfx950 Sternheimer library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>

namespace stern {

template <class T>
struct alignas(2 * sizeof(T)) Z {
  T re, im;
};
using Z64 = Z<double>;
using Z32 = Z<float>;

template <class T>
__host__ __device__ __forceinline__ Z<T> zmk(T a, T b) {
  Z<T> r;
  r.re = a;
  r.im = b;
  return r;
}
template <class T>
__host__ __device__ __forceinline__ Z<T> operator+(Z<T> a, Z<T> b) { return zmk(a.re + b.re, a.im + b.im); }
template <class T>
__host__ __device__ __forceinline__ Z<T> operator-(Z<T> a, Z<T> b) { return zmk(a.re - b.re, a.im - b.im); }
template <class T>
__host__ __device__ __forceinline__ Z<T> operator*(Z<T> a, Z<T> b) {
  return zmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__host__ __device__ __forceinline__ Z<T> zscale(Z<T> a, T s) { return zmk(a.re * s, a.im * s); }
template <class T>
__host__ __device__ __forceinline__ Z<T> zconj(Z<T> a) { return zmk(a.re, -a.im); }
// multiply by dir * i  (dir = +1 or -1)
template <int DIR, class T>
__host__ __device__ __forceinline__ Z<T> zmuli(Z<T> a) {
  return DIR > 0 ? zmk(-a.im, a.re) : zmk(a.im, -a.re);
}

// ---- compile-time cos/sin of 2 pi m / R (Taylor series after reduction to [-pi, pi]) ----
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double ct_sin_series(double x) {
  double x2 = x * x, term = x, s = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    s += term;
  }
  return s;
}
constexpr double ct_cos_series(double x) {
  double x2 = x * x, term = 1.0, s = 1.0;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    s += term;
  }
  return s;
}
// angle 2 pi m / R reduced to (-pi, pi], then folded into [-pi/2, pi/2] for the series
constexpr double ct_cos_frac(int m, int R) {
  int mm = ((m % R) + R) % R;
  if (2 * mm > R) mm -= R;              // now -R/2 < mm <= R/2
  double a = 2.0 * kPi * double(mm) / double(R);
  if (a > kPi / 2) return -ct_cos_series(kPi - a);
  if (a < -kPi / 2) return -ct_cos_series(-kPi - a);
  return ct_cos_series(a);
}
constexpr double ct_sin_frac(int m, int R) {
  int mm = ((m % R) + R) % R;
  if (2 * mm > R) mm -= R;
  double a = 2.0 * kPi * double(mm) / double(R);
  if (a > kPi / 2) return ct_sin_series(kPi - a);
  if (a < -kPi / 2) return ct_sin_series(-kPi - a);
  return ct_sin_series(a);
}

}  // namespace stern
