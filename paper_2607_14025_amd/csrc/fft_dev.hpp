// Device FFT building blocks: register DFTs of radix 2..16 and a batched
// two-stage Stockham FFT over lines held in LDS.
#pragma once
#include "common.hpp"

namespace stern {

// Two-stage plan N = R1 * R2 for every supported grid (2^a 3^b, 8..128).
template <int N>
struct Plan;
#define STERN_PLAN(N_, A_, B_)             \
  template <>                              \
  struct Plan<N_> {                        \
    static constexpr int R1 = A_, R2 = B_; \
  };
STERN_PLAN(8, 8, 1)
STERN_PLAN(9, 9, 1)
STERN_PLAN(12, 12, 1)
STERN_PLAN(16, 16, 1)
STERN_PLAN(18, 6, 3)
STERN_PLAN(24, 8, 3)
STERN_PLAN(27, 9, 3)
STERN_PLAN(32, 8, 4)
STERN_PLAN(36, 9, 4)
STERN_PLAN(48, 8, 6)
STERN_PLAN(54, 9, 6)
STERN_PLAN(64, 8, 8)
STERN_PLAN(72, 9, 8)
STERN_PLAN(81, 9, 9)
STERN_PLAN(96, 12, 8)
STERN_PLAN(108, 12, 9)
STERN_PLAN(128, 16, 8)
#undef STERN_PLAN

// Factorisation used for the in-register composite radices.
template <int R>
struct Split;
template <>
struct Split<6> { static constexpr int A = 3, B = 2; };
template <>
struct Split<8> { static constexpr int A = 4, B = 2; };
template <>
struct Split<9> { static constexpr int A = 3, B = 3; };
template <>
struct Split<12> { static constexpr int A = 4, B = 3; };
template <>
struct Split<16> { static constexpr int A = 4, B = 4; };

// v * exp(DIR * 2 pi i m / R), with exact handling of multiples of a quarter turn.
template <int R, int DIR, int M, class T>
__device__ __forceinline__ Z<T> rot_const(Z<T> v) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr ((4 * m) % R == 0) {
    constexpr int q = (4 * m) / R;  // quarter turns
    if constexpr (q == 1) return zmuli<DIR>(v);
    else if constexpr (q == 2) return zmk(-v.re, -v.im);
    else return zmuli<-DIR>(v);
  } else {
    constexpr T c = T(ct_cos_frac(m, R));
    constexpr T s = T(DIR * ct_sin_frac(m, R));
    return zmk(v.re * c - v.im * s, v.re * s + v.im * c);
  }
}

template <int R, int DIR, class T>
__device__ __forceinline__ void dft(Z<T>* v);

template <int DIR, class T>
__device__ __forceinline__ void dft2(Z<T>* v) {
  Z<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}
template <int DIR, class T>
__device__ __forceinline__ void dft3(Z<T>* v) {
  const T h = T(0.86602540378443864676372317075293618);
  Z<T> t = v[1] + v[2];
  Z<T> u = v[1] - v[2];
  Z<T> m = v[0] - zscale(t, T(0.5));
  Z<T> iu = zmuli<DIR>(zscale(u, h));
  v[0] = v[0] + t;
  v[1] = m + iu;
  v[2] = m - iu;
}
template <int DIR, class T>
__device__ __forceinline__ void dft4(Z<T>* v) {
  Z<T> a = v[0] + v[2], b = v[0] - v[2];
  Z<T> c = v[1] + v[3], d = zmuli<DIR>(v[1] - v[3]);
  v[0] = a + c;
  v[2] = a - c;
  v[1] = b + d;
  v[3] = b - d;
}

template <int R, int DIR, int A, int N2, class T, int... K1>
__device__ __forceinline__ void tw_row(const Z<T>* s, Z<T>* y, std::integer_sequence<int, K1...>) {
  ((y[N2 * A + K1] = rot_const<R, DIR, N2 * K1>(s[K1])), ...);
}

template <int A, int B, int DIR, class T, int N2>
__device__ __forceinline__ void composite_first(const Z<T>* v, Z<T>* y) {
  Z<T> s[A];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) s[n1] = v[N2 + B * n1];
  dft<A, DIR>(s);
  tw_row<A * B, DIR, A, N2>(s, y, std::make_integer_sequence<int, A>{});
}

template <int A, int B, int DIR, class T, int... N2>
__device__ __forceinline__ void composite_all_first(const Z<T>* v, Z<T>* y, std::integer_sequence<int, N2...>) {
  (composite_first<A, B, DIR, T, N2>(v, y), ...);
}

// R = A * B in registers: B DFTs of size A, twiddles exp(DIR 2 pi i n2 k1 / R), A DFTs of size B.
template <int A, int B, int DIR, class T>
__device__ __forceinline__ void dft_composite(Z<T>* v) {
  Z<T> y[A * B];
  composite_all_first<A, B, DIR, T>(v, y, std::make_integer_sequence<int, B>{});
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    Z<T> s[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) s[n2] = y[n2 * A + k1];
    dft<B, DIR>(s);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = s[k2];
  }
}

template <int R, int DIR, class T>
__device__ __forceinline__ void dft(Z<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<DIR>(v);
  } else if constexpr (R == 3) {
    dft3<DIR>(v);
  } else if constexpr (R == 4) {
    dft4<DIR>(v);
  } else {
    dft_composite<Split<R>::A, Split<R>::B, DIR>(v);
  }
}

// exp(DIR * 2 pi i m / N) from a table tw[m] = exp(-2 pi i m / N).
template <int DIR, class T>
__device__ __forceinline__ Z<T> twid(const Z<T>* __restrict__ tw, int m) {
  Z<T> w = tw[m];
  return DIR < 0 ? w : zconj(w);
}

struct NoPost {
  template <class T>
  __device__ __forceinline__ Z<T> operator()(int, int, int, int, Z<T> v) const { return v; }
};

// F independent length-N DFTs (sign DIR, unnormalised) of lines stored in LDS:
// element n of line f is buf[base(f) + n * stride]. Two Stockham stages
// (radix R1 then R2); stage 1 stages all of its items in registers before a
// barrier so it can run in place. The stage-2 store goes through
// post(f, n, slot, r, value), where slot is the item slot of this thread, so a
// caller can fuse a pointwise operation or keep per-thread accumulators.
// Ends with a barrier. Requires F <= MAXF.
template <int N, int DIR, int NT, int MAXF, class T, class Base, class Post>
__device__ __forceinline__ void fft_lines(Z<T>* buf, int F, int stride, Base base, Post post,
                                          const Z<T>* __restrict__ tw) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  const int tid = threadIdx.x;
  if constexpr (R2 == 1) {
    constexpr int MAXIT = (MAXF + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int f = tid + k * NT;
      if (f < F) {
        Z<T> v[R1];
        const int b0 = base(f);
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = buf[b0 + r * stride];
        dft<R1, DIR>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[b0 + r * stride] = post(f, r, k, r, v[r]);
      }
    }
    __syncthreads();
  } else {
    constexpr int MAXIT1 = (MAXF * R2 + NT - 1) / NT;
    Z<T> v[MAXIT1][R1];
#pragma unroll
    for (int k = 0; k < MAXIT1; ++k) {
      const int it = tid + k * NT;
      if (it < F * R2) {
        const int f = it / R2, j = it - f * R2;
        const int b0 = base(f);
#pragma unroll
        for (int r = 0; r < R1; ++r) v[k][r] = buf[b0 + (j + r * R2) * stride];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXIT1; ++k) {
      const int it = tid + k * NT;
      if (it < F * R2) {
        const int f = it / R2, j = it - f * R2;
        const int b0 = base(f);
        dft<R1, DIR>(v[k]);
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[b0 + (j * R1 + r) * stride] = v[k][r];
      }
    }
    __syncthreads();
    constexpr int MAXIT2 = (MAXF * R1 + NT - 1) / NT;
#pragma unroll
    for (int k = 0; k < MAXIT2; ++k) {
      const int it = tid + k * NT;
      if (it < F * R1) {
        const int f = it / R1, j = it - f * R1;
        const int b0 = base(f);
        Z<T> w[R2];
        w[0] = buf[b0 + j * stride];
#pragma unroll
        for (int r = 1; r < R2; ++r) w[r] = buf[b0 + (j + r * R1) * stride] * twid<DIR>(tw, r * j);
        dft<R2, DIR>(w);
#pragma unroll
        for (int r = 0; r < R2; ++r) buf[b0 + (j + r * R1) * stride] = post(f, j + r * R1, k, r, w[r]);
      }
    }
    __syncthreads();
  }
}

}  // namespace stern
