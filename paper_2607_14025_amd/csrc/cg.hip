// Per-solve vector kernels of the projected PCG: one workgroup per solve,
// FP64 scalars and FP64 dot products with a fixed reduction order (so runs are
// bitwise reproducible), Teter-Payne-Allan diagonal preconditioner
//   K(G) = (27 + 18y + 12y^2 + 8y^3) / (27 + 18y + 12y^2 + 8y^3 + 16y^4), y = (|G|^2/2) / T_v
// (Phys. Rev. B 40, 12255 (1989)) evaluated on the fly.
#include "kernels.hpp"

namespace stern {

namespace {

constexpr int kCgThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kCgThreads / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ double teter(double g2h, double invT) {
  const double y = g2h * invT;
  const double num = 27.0 + y * (18.0 + y * (12.0 + 8.0 * y));
  const double y2 = y * y;
  return num / (num + 16.0 * y2 * y2);
}

// diagonal preconditioner of solve s at coefficient k: the learned K when given, else Teter
template <class St>
__device__ __forceinline__ double precond(const St& S, int s, int k, double iT) {
  return S.kprec ? (double)S.kprec[(size_t)s * S.npw_pad + k] : teter(S.g2h[k], iT);
}
// the same in two steps, so that the load can be issued with the vector loads; LK: the
// learned K is given (a launch-wide choice, a template parameter so no branch splits the loads)
template <bool LK, class St>
__device__ __forceinline__ double precond_load(const St& S, int s, int k) {
  if constexpr (LK) return (double)S.kprec[(size_t)s * S.npw_pad + k];
  else return S.g2h[k];
}
template <bool LK>
__device__ __forceinline__ double precond_eval(double raw, double iT) {
  if constexpr (LK) return raw;
  else return teter(raw, iT);
}

// The vector loops below take kU coefficients per thread per trip, all loaded before
// any is used (kU independent loads in flight instead of one). A thread still visits
// k = tid, tid + kCgThreads, tid + 2 kCgThreads, ... in order, so every FP64 sum has
// the order of the one-at-a-time loop.
constexpr int kU = 4;

// keep == 0: x = 0, r = b. keep != 0: x and r = b - A x are given (a guess).
// z = K r; ||b||^2; flag 0 (2 when b = 0).
__global__ __launch_bounds__(kCgThreads) void k_cg_init(CgState S, const int* __restrict__ act, int keep) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  const double iT = S.invT[s];
  double bb = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 b = S.b[o + k];
    bb += b.re * b.re + b.im * b.im;
    Z64 r = b;
    if (keep) {
      r = S.r[o + k];
    } else {
      S.x[o + k] = zmk(0.0, 0.0);
      S.r[o + k] = b;
    }
    S.z[o + k] = zscale(r, precond(S, s, k, iT));
  }
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    S.bb[s] = bb;
    S.flag[s] = (bb > 0.0) ? 0 : 2;
  }
}

// r = b - q + i u x for a guess x, with q = P_c (H - eps) P_c x given in FP64 (q32 == null) or
// FP32 and u the imaginary frequency (0: the static system); the guess is kept only if ||r|| is
// finite and below ||b|| by more than rounding (||r||^2 < (1 - 2^-40) ||b||^2: a zero guess, whose
// ||r||^2 differs from ||b||^2 only by the order of the two sums, is always rejected), else
// x = 0, r = b. With tol2 >= 0 a kept guess with ||r||^2 <= tol2 ||b||^2 is a converged solve
// (flag 2, no iteration).
__global__ __launch_bounds__(kCgThreads) void k_guess_resid(CgState S, const int* __restrict__ act,
                                                            const Z32* __restrict__ q32, int* __restrict__ rejected,
                                                            double u, double tol2) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  auto res = [&](int k) -> Z64 {
    Z64 q;
    if (q32) {
      const Z32 v = q32[o + k];
      q = zmk((double)v.re, (double)v.im);
    } else {
      q = S.q[o + k];
    }
    const Z64 b = S.b[o + k], x = S.x[o + k];
    return zmk(b.re - q.re - u * x.im, b.im - q.im + u * x.re);
  };
  double rr = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 r = res(k);
    rr += r.re * r.re + r.im * r.im;
  }
  rr = block_sum(rr, sh);
  const bool ok = (rr == rr) && rr < (1.0 - 0x1p-40) * S.bb[s];  // false for NaN
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    if (ok) {
      S.r[o + k] = res(k);
    } else {
      S.r[o + k] = S.b[o + k];
      S.x[o + k] = zmk(0.0, 0.0);
    }
  }
  if (threadIdx.x == 0) {
    const bool zero_b = !(S.bb[s] > 0.0);  // b = 0: x = 0 is exact, nothing was rejected
    rejected[s] = (ok || zero_b) ? 0 : 1;
    S.tres[s] = ok ? sqrt(rr / S.bb[s]) : (zero_b ? 0.0 : 1.0);
    if (ok && tol2 >= 0.0 && rr <= tol2 * S.bb[s]) S.flag[s] = 2;
  }
}

// y = (float) x on rows [0, n) of length ld
__global__ void k_to32(const Z64* __restrict__ x, Z32* __restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const Z64 v = x[i];
    y[i] = zmk((float)v.re, (float)v.im);
  }
}

__global__ __launch_bounds__(kCgThreads) void k_cg_init2(CgState S, const int* __restrict__ act) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  double rz = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 r = S.r[o + k], z = S.z[o + k];
    rz += r.re * z.re + r.im * z.im;
    S.p[o + k] = z;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) S.rz[s] = rz;
}

// alpha = <r,z> / <p,q>; x += alpha p; r -= alpha q; z = K r; flag on ||r|| <= tol ||b||
template <bool LK>
__global__ __launch_bounds__(kCgThreads) void k_cg_alpha(CgState S, const int* __restrict__ act, double tol2) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const int n = S.npw_pad;
  double pq = 0.0;
  for (int k0 = threadIdx.x; k0 < n; k0 += kCgThreads * kU) {
    Z64 p[kU], q[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        p[u] = S.p[o + k];
        q[u] = S.q[o + k];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k0 + u * kCgThreads < n) pq += p[u].re * q[u].re + p[u].im * q[u].im;
  }
  pq = block_sum(pq, sh);
  const double alpha = (pq > 0.0) ? S.rz[s] / pq : 0.0;
  const double iT = S.invT[s];
  double rr = 0.0;
  for (int k0 = threadIdx.x; k0 < n; k0 += kCgThreads * kU) {
    Z64 p[kU], q[kU], x[kU], r[kU];
    double t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        p[u] = S.p[o + k];
        q[u] = S.q[o + k];
        x[u] = S.x[o + k];
        r[u] = S.r[o + k];
        t[u] = precond_load<LK>(S, s, k);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        const Z64 xn = zmk(x[u].re + alpha * p[u].re, x[u].im + alpha * p[u].im);
        const Z64 rn = zmk(r[u].re - alpha * q[u].re, r[u].im - alpha * q[u].im);
        S.x[o + k] = xn;
        S.r[o + k] = rn;
        rr += rn.re * rn.re + rn.im * rn.im;
        S.z[o + k] = zscale(rn, precond_eval<LK>(t[u], iT));
      }
    }
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    S.rr[s] = rr;
    S.iters[s] += 1;
    if (rr <= tol2 * S.bb[s] || !(pq > 0.0)) S.flag[s] = 1;
  }
}

// beta = <r,z>_new / <r,z>_old; p = z + beta p
__global__ __launch_bounds__(kCgThreads) void k_cg_beta(CgState S, const int* __restrict__ act) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const int n = S.npw_pad;
  double rz = 0.0;
  for (int k0 = threadIdx.x; k0 < n; k0 += kCgThreads * kU) {
    Z64 r[kU], z[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        r[u] = S.r[o + k];
        z[u] = S.z[o + k];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k0 + u * kCgThreads < n) rz += r[u].re * z[u].re + r[u].im * z[u].im;
  }
  rz = block_sum(rz, sh);
  const double beta = rz / S.rz[s];
  for (int k0 = threadIdx.x; k0 < n; k0 += kCgThreads * kU) {
    Z64 z[kU], p[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        z[u] = S.z[o + k];
        p[u] = S.p[o + k];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) S.p[o + k] = zmk(z[u].re + beta * p[u].re, z[u].im + beta * p[u].im);
    }
  }
  if (threadIdx.x == 0) S.rz[s] = rz;
}

__global__ void k_copy_rows(const Z64* __restrict__ src, Z64* __restrict__ dst, int ld, const int* __restrict__ act) {
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * ld;
  for (int k = threadIdx.x; k < ld; k += blockDim.x) dst[o + k] = src[o + k];
}

// q holds A x for solves with flag 1: accept (flag 2) or restart from r = b - A x (flag 3)
__global__ __launch_bounds__(kCgThreads) void k_true_resid(CgState S, const int* __restrict__ act, double tol) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 1) return;
  const size_t o = (size_t)s * S.npw_pad;
  double tt = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 b = S.b[o + k], q = S.q[o + k];
    const double re = b.re - q.re, im = b.im - q.im;
    tt += re * re + im * im;
  }
  tt = block_sum(tt, sh);
  const double bb = S.bb[s];
  const bool ok = tt <= tol * tol * bb;
  if (!ok) {
    const double iT = S.invT[s];
    for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
      const Z64 b = S.b[o + k], q = S.q[o + k];
      const Z64 r = zmk(b.re - q.re, b.im - q.im);
      S.r[o + k] = r;
      S.z[o + k] = zscale(r, precond(S, s, k, iT));
    }
  }
  if (threadIdx.x == 0) {
    S.tres[s] = sqrt(tt / bb);
    S.flag[s] = ok ? 2 : 3;
  }
}

__global__ __launch_bounds__(kCgThreads) void k_cg_restart(CgState S, const int* __restrict__ act) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 3) return;
  const size_t o = (size_t)s * S.npw_pad;
  double rz = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 r = S.r[o + k], z = S.z[o + k];
    rz += r.re * z.re + r.im * z.im;
    S.p[o + k] = z;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    S.rz[s] = rz;
    S.flag[s] = 0;
  }
}

__global__ void k_permute(const Z64* __restrict__ in, int ld_in, Z64* __restrict__ out, int ld_out,
                          const int* __restrict__ perm, int npw, int scatter) {
  const int v = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npw) return;
  if (scatter)
    out[(size_t)v * ld_out + perm[k]] = in[(size_t)v * ld_in + k];
  else
    out[(size_t)v * ld_out + k] = in[(size_t)v * ld_in + perm[k]];
}

__global__ void k_fill_zero(Z64* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = zmk(0.0, 0.0);
}

__global__ void k_set_flag(int* __restrict__ flag, const int* __restrict__ list, int n, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[list[i]] = value;
}

// complex field from a real one (zero imaginary part), and the real part of a complex one times scale
__global__ void k_real_to_z(const double* __restrict__ in, Z64* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = zmk(in[i], 0.0);
}
__global__ void k_z_real(const Z64* __restrict__ in, double scale, double* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = scale * in[i].re;
}

__global__ void k_ri(const double* __restrict__ in, Z64* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = zmk(in[2 * i], in[2 * i + 1]);
}

// ---------------------------------------------------------------- mixed ----
// FP32 inner CG of the defect correction: vectors in FP32, dots accumulated
// and scalars kept in FP64.

// ri = fp32(r64); d = 0; z = K ri; rr0 = ||ri||^2; inner flag 0 (2 if rr0 == 0)
__global__ __launch_bounds__(kCgThreads) void k_cg32_init(Cg32State S, const Z64* __restrict__ r64,
                                                          const int* __restrict__ act) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  const double iT = S.invT[s];
  double rr = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 v = r64[o + k];
    const Z32 r = zmk((float)v.re, (float)v.im);
    rr += (double)r.re * r.re + (double)r.im * r.im;
    S.r[o + k] = r;
    S.d[o + k] = zmk(0.f, 0.f);
    const float t = (float)precond(S, s, k, iT);
    S.z[o + k] = zmk(r.re * t, r.im * t);
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    S.rr0[s] = rr;
    S.flag[s] = rr > 0.0 ? 0 : 2;
  }
}

__global__ __launch_bounds__(kCgThreads) void k_cg32_init2(Cg32State S, const int* __restrict__ act) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  double rz = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z32 r = S.r[o + k], z = S.z[o + k];
    rz += (double)r.re * z.re + (double)r.im * z.im;
    S.p[o + k] = z;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) S.rz[s] = rz;
}

// alpha = (r, z) / (p, q); d += alpha p; r -= alpha q; z = K r; the new (r, z)
// and beta = (r, z) new / old for the direction update that follows; inner
// flag 1 once ||r||^2 <= tol2 ||r0||^2. (r, z) is taken with z before any
// projection: r stays in range(P_c), so it equals (r, P_c z).
template <bool LK>
__global__ __launch_bounds__(kCgThreads) void k_cg32_alpha(Cg32State S, const int* __restrict__ act, double tol2,
                                                             const int* __restrict__ live) {
  __shared__ double sh[kCgThreads / 64];
  if (live && (int)blockIdx.x >= *live) return;  // list entry past the live count (whole workgroup)
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const int n = S.npw_pad;
  double pq = 0.0;
  for (int k0 = threadIdx.x; k0 < n; k0 += kCgThreads * kU) {
    Z32 p[kU], q[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        p[u] = S.p[o + k];
        q[u] = S.q[o + k];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k0 + u * kCgThreads < n) pq += (double)p[u].re * q[u].re + (double)p[u].im * q[u].im;
  }
  pq = block_sum(pq, sh);
  const double rz_old = S.rz[s];
  const float alpha = (float)((pq > 0.0) ? rz_old / pq : 0.0);
  const double iT = S.invT[s];
  double rr = 0.0, rz = 0.0;
  for (int k0 = threadIdx.x; k0 < n; k0 += kCgThreads * kU) {
    Z32 p[kU], q[kU], d[kU], r[kU];
    double t[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        p[u] = S.p[o + k];
        q[u] = S.q[o + k];
        d[u] = S.d[o + k];
        r[u] = S.r[o + k];
        t[u] = precond_load<LK>(S, s, k);
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * kCgThreads;
      if (k < n) {
        const Z32 dn = zmk(d[u].re + alpha * p[u].re, d[u].im + alpha * p[u].im);
        const Z32 rn = zmk(r[u].re - alpha * q[u].re, r[u].im - alpha * q[u].im);
        S.d[o + k] = dn;
        S.r[o + k] = rn;
        rr += (double)rn.re * rn.re + (double)rn.im * rn.im;
        const float tk = (float)precond_eval<LK>(t[u], iT);
        const Z32 z = zmk(rn.re * tk, rn.im * tk);
        S.z[o + k] = z;
        rz += (double)rn.re * z.re + (double)rn.im * z.im;
      }
    }
  }
  rr = block_sum(rr, sh);
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    S.iters[s] += 1;
    if (rr <= tol2 * S.rr0[s] || !(pq > 0.0)) S.flag[s] = 1;
    S.beta[s] = rz_old != 0.0 ? rz / rz_old : 0.0;
    S.rz[s] = rz;
  }
}

// The alpha step above with the whole row in one workgroup of kAlphaThreads: each thread
// keeps its PER elements of p and q in registers from the (p, q) sum to the update, so p
// and q are read once instead of twice. For rows up to kAlphaThreads * PER elements
// (PER <= 17 keeps p and q within 68 VGPRs, four waves per SIMD).
constexpr int kAlphaThreads = 1024;
constexpr int kAlphaMaxPer = 17;

__device__ __forceinline__ double block_sum_a(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kAlphaThreads / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

template <bool LK, int PER>
__global__ __launch_bounds__(kAlphaThreads) void k_cg32_alpha_row(Cg32State S, const int* __restrict__ act,
                                                                   double tol2, const int* __restrict__ live) {
  __shared__ double sh[kAlphaThreads / 64];
  if (live && (int)blockIdx.x >= *live) return;  // list entry past the live count (whole workgroup)
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const int n = S.npw_pad;
  Z32 p[PER], q[PER];
  double pq = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int k = threadIdx.x + u * kAlphaThreads;
    if (k < n) {
      p[u] = S.p[o + k];
      q[u] = S.q[o + k];
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u)
    if (threadIdx.x + u * kAlphaThreads < n) pq += (double)p[u].re * q[u].re + (double)p[u].im * q[u].im;
  pq = block_sum_a(pq, sh);
  const double rz_old = S.rz[s];
  const float alpha = (float)((pq > 0.0) ? rz_old / pq : 0.0);
  const double iT = S.invT[s];
  double rr = 0.0, rz = 0.0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int k = threadIdx.x + u * kAlphaThreads;
    if (k < n) {
      const Z32 d = S.d[o + k], r = S.r[o + k];
      const double t = precond_load<LK>(S, s, k);
      const Z32 dn = zmk(d.re + alpha * p[u].re, d.im + alpha * p[u].im);
      const Z32 rn = zmk(r.re - alpha * q[u].re, r.im - alpha * q[u].im);
      S.d[o + k] = dn;
      S.r[o + k] = rn;
      rr += (double)rn.re * rn.re + (double)rn.im * rn.im;
      const float tk = (float)precond_eval<LK>(t, iT);
      const Z32 z = zmk(rn.re * tk, rn.im * tk);
      S.z[o + k] = z;
      rz += (double)rn.re * z.re + (double)rn.im * z.im;
    }
  }
  rr = block_sum_a(rr, sh);
  rz = block_sum_a(rz, sh);
  if (threadIdx.x == 0) {
    S.iters[s] += 1;
    if (rr <= tol2 * S.rr0[s] || !(pq > 0.0)) S.flag[s] = 1;
    S.beta[s] = rz_old != 0.0 ? rz / rz_old : 0.0;
    S.rz[s] = rz;
  }
}

// p = z + beta p (beta from the alpha step)
__global__ __launch_bounds__(kCgThreads) void k_cg32_beta(Cg32State S, const int* __restrict__ act,
                                                            const int* __restrict__ live) {
  if (live && (int)blockIdx.x >= *live) return;  // list entry past the live count (whole workgroup)
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const float beta = (float)S.beta[s];
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z32 z = S.z[o + k], p = S.p[o + k];
    S.p[o + k] = zmk(z.re + beta * p.re, z.im + beta * p.im);
  }
}

// x64 += d32
__global__ void k_add_d(Z64* __restrict__ x, const Z32* __restrict__ d, int ld, const int* __restrict__ act) {
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * ld;
  for (int k = threadIdx.x; k < ld; k += blockDim.x) {
    const Z64 a = x[o + k];
    const Z32 b = d[o + k];
    x[o + k] = zmk(a.re + (double)b.re, a.im + (double)b.im);
  }
}

// r = b - q (FP64 true residual of the outer loop); accept when ||r|| <= tol ||b||
__global__ __launch_bounds__(kCgThreads) void k_outer_resid(CgState S, const int* __restrict__ act, double tol) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  double tt = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 b = S.b[o + k], q = S.q[o + k];
    const Z64 r = zmk(b.re - q.re, b.im - q.im);
    S.r[o + k] = r;
    tt += r.re * r.re + r.im * r.im;
  }
  tt = block_sum(tt, sh);
  if (threadIdx.x == 0) {
    const double bb = S.bb[s];
    S.tres[s] = bb > 0.0 ? sqrt(tt / bb) : 0.0;
    S.flag[s] = (tt <= tol * tol * bb) ? 2 : 0;
  }
}

// x = 0, r = b, bb = ||b||^2 (outer loop start); flag 2 when b = 0
// bb[s] = ||y_s||^2 over one row (the right-hand side before its projection).
__global__ __launch_bounds__(kCgThreads) void k_row_norm2(const Z64* __restrict__ y, int ld, double* __restrict__ out) {
  __shared__ double sh[kCgThreads / 64];
  const size_t o = (size_t)blockIdx.x * ld;
  double t = 0.0;
  for (int k = threadIdx.x; k < ld; k += kCgThreads) {
    const Z64 v = y[o + k];
    t += v.re * v.re + v.im * v.im;
  }
  t = block_sum(t, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// x = 0, r = b, counters. S.bb holds ||dV psi_v||^2 of the unprojected product on entry:
// a projected b with ||b||^2 <= cut2 ||dV psi_v||^2 is rounding left by the projection
// of a product that lies in the occupied span, and is set to zero (x = 0, done).
__global__ __launch_bounds__(kCgThreads) void k_outer_init(CgState S, const int* __restrict__ act, double cut2) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  const size_t o = (size_t)s * S.npw_pad;
  const double raw = S.bb[s];
  double bb = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 b = S.b[o + k];
    bb += b.re * b.re + b.im * b.im;
    S.x[o + k] = zmk(0.0, 0.0);
    S.r[o + k] = b;
  }
  bb = block_sum(bb, sh);
  if (bb <= cut2 * raw) {
    for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
      S.b[o + k] = zmk(0.0, 0.0);
      S.r[o + k] = zmk(0.0, 0.0);
    }
    bb = 0.0;
  }
  if (threadIdx.x == 0) {
    S.bb[s] = bb;
    S.iters[s] = 0;
    S.tres[s] = bb > 0.0 ? 1.0 : 0.0;
    S.flag[s] = bb > 0.0 ? 0 : 2;
  }
}

__global__ void k_fill_zero32(Z32* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = zmk(0.f, 0.f);
}

// ---- conjugate orthogonal CG for the shifted systems of the response at imaginary frequency ----
//
// (P_c (H - eps_v) P_c - i u) x = b on range(P_c). The shifted operator is not Hermitian, but it
// is symmetric in the bilinear form (a, b)_J = sum_G a(-G) b(G): H commutes with the map
// a(G) -> conj a(-G) (a real local potential and projectors whose radial parts are real), so
// does the projector on a complete occupied subspace of such an H, and so do the identity and
// a preconditioner that depends on |G| only; an operator that commutes with that map is
// symmetric in (., .)_J. Conjugate orthogonal CG (van der Vorst and Melissen, IEEE Trans. Magn.
// 26, 706 (1990)) is CG with (., .)_J in place of the inner product: one operator apply per
// iteration and complex scalars. negk[k] is the index of -G for the coefficient k (column
// order; the padding maps to itself). The complex rho = (r, z)_J of solve s is (rz[s], rzi[s]).

__device__ __forceinline__ Z64 block_sum_z(Z64 v, double* sh) {
  const double re = block_sum(v.re, sh);
  const double im = block_sum(v.im, sh);
  return zmk(re, im);
}
__device__ __forceinline__ Z64 zdiv(Z64 a, Z64 b) {
  const double d = b.re * b.re + b.im * b.im;
  return zmk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

// p = z; rho = (r, z)_J, for solves whose flag equals `from` (0: start, 3: restart); flag -> 0
__global__ __launch_bounds__(kCgThreads) void k_cocg_start(CgState S, const int* __restrict__ negk,
                                                           double* __restrict__ rzi, const int* __restrict__ act,
                                                           int from) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != from) return;
  const size_t o = (size_t)s * S.npw_pad;
  Z64 rz = zmk(0.0, 0.0);
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 r = S.r[o + negk[k]], z = S.z[o + k];
    rz = rz + r * z;
    S.p[o + k] = z;
  }
  rz = block_sum_z(rz, sh);
  if (threadIdx.x == 0) {
    S.rz[s] = rz.re;
    rzi[s] = rz.im;
    S.flag[s] = 0;
  }
}

// q holds P_c (H - eps) P_c p; with qs = q - i u p: alpha = rho / (p, qs)_J; x += alpha p;
// r -= alpha qs; z = K r; flag 1 on ||r|| <= tol ||b|| (or a vanishing (p, qs)_J)
template <bool LK>
__global__ __launch_bounds__(kCgThreads) void k_cocg_alpha(CgState S, const int* __restrict__ negk,
                                                           const double* __restrict__ rzi, double u,
                                                           const int* __restrict__ act, double tol2) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const int n = S.npw_pad;
  Z64 pq = zmk(0.0, 0.0);
  for (int k = threadIdx.x; k < n; k += kCgThreads) {
    const Z64 p = S.p[o + k], q = S.q[o + k], pm = S.p[o + negk[k]];
    pq = pq + pm * zmk(q.re + u * p.im, q.im - u * p.re);  // q - i u p
  }
  pq = block_sum_z(pq, sh);
  const bool ok = pq.re != 0.0 || pq.im != 0.0;
  const Z64 alpha = ok ? zdiv(zmk(S.rz[s], rzi[s]), pq) : zmk(0.0, 0.0);
  const double iT = S.invT[s];
  double rr = 0.0;
  for (int k = threadIdx.x; k < n; k += kCgThreads) {
    const Z64 p = S.p[o + k], q = S.q[o + k];
    const Z64 qs = zmk(q.re + u * p.im, q.im - u * p.re);
    const Z64 xn = S.x[o + k] + alpha * p;
    const Z64 rn = S.r[o + k] - alpha * qs;
    S.x[o + k] = xn;
    S.r[o + k] = rn;
    rr += rn.re * rn.re + rn.im * rn.im;
    S.z[o + k] = zscale(rn, precond_eval<LK>(precond_load<LK>(S, s, k), iT));
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    S.rr[s] = rr;
    S.iters[s] += 1;
    if (rr <= tol2 * S.bb[s] || !ok) S.flag[s] = 1;
  }
}

// beta = (r, z)_J new / old; p = z + beta p
__global__ __launch_bounds__(kCgThreads) void k_cocg_beta(CgState S, const int* __restrict__ negk,
                                                          double* __restrict__ rzi, const int* __restrict__ act) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 0) return;
  const size_t o = (size_t)s * S.npw_pad;
  const int n = S.npw_pad;
  Z64 rz = zmk(0.0, 0.0);
  for (int k = threadIdx.x; k < n; k += kCgThreads) rz = rz + S.r[o + negk[k]] * S.z[o + k];
  rz = block_sum_z(rz, sh);
  const Z64 beta = zdiv(rz, zmk(S.rz[s], rzi[s]));
  for (int k = threadIdx.x; k < n; k += kCgThreads) S.p[o + k] = S.z[o + k] + beta * S.p[o + k];
  if (threadIdx.x == 0) {
    S.rz[s] = rz.re;
    rzi[s] = rz.im;
  }
}

// For solves with flag 1: z holds P_c x and q holds P_c (H - eps) P_c x. The true residual
// b - (q - i u z) is accepted (flag 2) or becomes the new r with z = K r (flag 3: restart)
__global__ __launch_bounds__(kCgThreads) void k_cocg_true(CgState S, double u, const int* __restrict__ act,
                                                          double tol) {
  __shared__ double sh[kCgThreads / 64];
  const int s = act ? act[blockIdx.x] : blockIdx.x;
  if (S.flag[s] != 1) return;
  const size_t o = (size_t)s * S.npw_pad;
  double tt = 0.0;
  for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
    const Z64 b = S.b[o + k], q = S.q[o + k], x = S.z[o + k];
    const double re = b.re - q.re - u * x.im, im = b.im - q.im + u * x.re;
    tt += re * re + im * im;
  }
  tt = block_sum(tt, sh);
  const double bb = S.bb[s];
  const bool ok = tt <= tol * tol * bb;
  if (!ok) {
    const double iT = S.invT[s];
    for (int k = threadIdx.x; k < S.npw_pad; k += kCgThreads) {
      const Z64 b = S.b[o + k], q = S.q[o + k], x = S.z[o + k];
      const Z64 r = zmk(b.re - q.re - u * x.im, b.im - q.im + u * x.re);
      S.r[o + k] = r;
      S.z[o + k] = zscale(r, precond(S, s, k, iT));
    }
  }
  if (threadIdx.x == 0) {
    S.tres[s] = sqrt(tt / bb);
    S.flag[s] = ok ? 2 : 3;
  }
}

// ---- block vectors of the Liouville solve: one block = the nb band rows of one excitation ----

// out[row] = sum_k conj(a[row][k]) b[row][k], fixed order
__global__ __launch_bounds__(kCgThreads) void k_row_dot(const Z64* __restrict__ a, const Z64* __restrict__ b, int ld,
                                                        Z64* __restrict__ out) {
  __shared__ double sh[kCgThreads / 64];
  const size_t o = (size_t)blockIdx.x * ld;
  Z64 d = zmk(0.0, 0.0);
  for (int k = threadIdx.x; k < ld; k += kCgThreads) {
    const Z64 x = a[o + k], y = b[o + k];
    d.re += x.re * y.re + x.im * y.im;
    d.im += x.re * y.im - x.im * y.re;
  }
  d = block_sum_z(d, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = d;
}

// y[row] += c[row / nb] x[row]
__global__ __launch_bounds__(kCgThreads) void k_blk_axpy(Z64* __restrict__ y, const Z64* __restrict__ x,
                                                         const Z64* __restrict__ c, int nb, int ld) {
  const Z64 a = c[blockIdx.x / nb];
  const size_t o = (size_t)blockIdx.x * ld;
  for (int k = threadIdx.x; k < ld; k += kCgThreads) {
    const Z64 v = x[o + k], w = y[o + k];
    y[o + k] = zmk(w.re + a.re * v.re - a.im * v.im, w.im + a.re * v.im + a.im * v.re);
  }
}

// p[row] = z[row] + c[row / nb] p[row]
__global__ __launch_bounds__(kCgThreads) void k_blk_xpby(Z64* __restrict__ p, const Z64* __restrict__ z,
                                                         const Z64* __restrict__ c, int nb, int ld) {
  const Z64 a = c[blockIdx.x / nb];
  const size_t o = (size_t)blockIdx.x * ld;
  for (int k = threadIdx.x; k < ld; k += kCgThreads) {
    const Z64 v = p[o + k], w = z[o + k];
    p[o + k] = zmk(w.re + a.re * v.re - a.im * v.im, w.im + a.re * v.im + a.im * v.re);
  }
}

// y[row] *= c[row / nb]
__global__ __launch_bounds__(kCgThreads) void k_blk_scale(Z64* __restrict__ y, const Z64* __restrict__ c, int nb,
                                                          int ld) {
  const Z64 a = c[blockIdx.x / nb];
  const size_t o = (size_t)blockIdx.x * ld;
  for (int k = threadIdx.x; k < ld; k += kCgThreads) {
    const Z64 w = y[o + k];
    y[o + k] = zmk(a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re);
  }
}

// z[row][k] = K_v(G) r[row][k], Teter's K with T_v of band v = row mod nb
__global__ __launch_bounds__(kCgThreads) void k_teter_rows(const Z64* __restrict__ r, Z64* __restrict__ z,
                                                           const double* __restrict__ g2h,
                                                           const double* __restrict__ invT, int nb, int ld) {
  const double iT = invT[blockIdx.x % nb];
  const size_t o = (size_t)blockIdx.x * ld;
  for (int k = threadIdx.x; k < ld; k += kCgThreads) z[o + k] = zscale(r[o + k], teter(g2h[k], iT));
}

}  // namespace

void launch_cocg_start(const CgState& s, const int* negk, double* rzi, const int* act, int n, int from,
                       hipStream_t st) {
  if (n > 0) k_cocg_start<<<n, kCgThreads, 0, st>>>(s, negk, rzi, act, from);
}
void launch_cocg_alpha(const CgState& s, const int* negk, const double* rzi, double u, const int* act, int n,
                       double tol2, hipStream_t st) {
  if (n <= 0) return;
  if (s.kprec)
    k_cocg_alpha<true><<<n, kCgThreads, 0, st>>>(s, negk, rzi, u, act, tol2);
  else
    k_cocg_alpha<false><<<n, kCgThreads, 0, st>>>(s, negk, rzi, u, act, tol2);
}
void launch_cocg_beta(const CgState& s, const int* negk, double* rzi, const int* act, int n, hipStream_t st) {
  if (n > 0) k_cocg_beta<<<n, kCgThreads, 0, st>>>(s, negk, rzi, act);
}
void launch_cocg_true(const CgState& s, double u, const int* act, int n, double tol, hipStream_t st) {
  if (n > 0) k_cocg_true<<<n, kCgThreads, 0, st>>>(s, u, act, tol);
}

void launch_cg_init(const CgState& s, const int* act, int n, bool keep, hipStream_t st) {
  if (n > 0) k_cg_init<<<n, kCgThreads, 0, st>>>(s, act, keep ? 1 : 0);
}
void launch_guess_resid(const CgState& s, const int* act, int n, const Z32* q32, int* rejected, hipStream_t st,
                        double u, double tol2) {
  if (n > 0) k_guess_resid<<<n, kCgThreads, 0, st>>>(s, act, q32, rejected, u, tol2);
}
void launch_to32(const Z64* x, Z32* y, size_t n, hipStream_t st) {
  if (n == 0) return;
  k_to32<<<(unsigned)std::min<size_t>((n + 255) / 256, 65536), 256, 0, st>>>(x, y, n);
}
void launch_cg_init2(const CgState& s, const int* act, int n, hipStream_t st) {
  if (n > 0) k_cg_init2<<<n, kCgThreads, 0, st>>>(s, act);
}
void launch_cg_alpha(const CgState& s, const int* act, int n, double tol2, hipStream_t st) {
  if (n <= 0) return;
  if (s.kprec)
    k_cg_alpha<true><<<n, kCgThreads, 0, st>>>(s, act, tol2);
  else
    k_cg_alpha<false><<<n, kCgThreads, 0, st>>>(s, act, tol2);
}
void launch_cg_beta(const CgState& s, const int* act, int n, hipStream_t st) {
  if (n > 0) k_cg_beta<<<n, kCgThreads, 0, st>>>(s, act);
}
void launch_copy_rows(const Z64* src, Z64* dst, int ld, const int* act, int n, hipStream_t st) {
  if (n > 0) k_copy_rows<<<n, 256, 0, st>>>(src, dst, ld, act);
}
void launch_true_resid(const CgState& s, const int* act, int n, double tol, hipStream_t st) {
  if (n > 0) k_true_resid<<<n, kCgThreads, 0, st>>>(s, act, tol);
}
void launch_cg_restart(const CgState& s, const int* act, int n, hipStream_t st) {
  if (n > 0) k_cg_restart<<<n, kCgThreads, 0, st>>>(s, act);
}
void launch_permute(const Z64* in, int ld_in, Z64* out, int ld_out, const int* perm, int npw, int nvec, bool scatter,
                    hipStream_t st) {
  if (nvec <= 0 || npw <= 0) return;
  dim3 grid((npw + 255) / 256, nvec);
  k_permute<<<grid, 256, 0, st>>>(in, ld_in, out, ld_out, perm, npw, scatter ? 1 : 0);
}
void launch_fill_zero(Z64* p, size_t n, hipStream_t st) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill_zero<<<(unsigned)blocks, 256, 0, st>>>(p, n);
}
void launch_set_flag(int* flag, const int* list, int n, int value, hipStream_t st) {
  if (n > 0) k_set_flag<<<(n + 255) / 256, 256, 0, st>>>(flag, list, n, value);
}
void launch_real_to_z(const double* in, Z64* out, size_t n, hipStream_t st) {
  if (n == 0) return;
  const size_t b = (n + 255) / 256;
  k_real_to_z<<<(unsigned)(b > 65536 ? 65536 : b), 256, 0, st>>>(in, out, n);
}
void launch_z_real(const Z64* in, double scale, double* out, size_t n, hipStream_t st) {
  if (n == 0) return;
  const size_t b = (n + 255) / 256;
  k_z_real<<<(unsigned)(b > 65536 ? 65536 : b), 256, 0, st>>>(in, scale, out, n);
}
void launch_ri_to_complex(const double* in, Z64* out, size_t n, hipStream_t st) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_ri<<<(unsigned)blocks, 256, 0, st>>>(in, out, n);
}

}  // namespace stern

namespace stern {
void launch_cg32_init(const Cg32State& s, const Z64* r64, const int* act, int n, hipStream_t st) {
  if (n > 0) k_cg32_init<<<n, kCgThreads, 0, st>>>(s, r64, act);
}
void launch_cg32_init2(const Cg32State& s, const int* act, int n, hipStream_t st) {
  if (n > 0) k_cg32_init2<<<n, kCgThreads, 0, st>>>(s, act);
}
void launch_cg32_alpha(const Cg32State& s, const int* act, int n, double tol2, hipStream_t st, const int* live) {
  if (n <= 0) return;
  if (s.npw_pad <= kAlphaThreads * kAlphaMaxPer) {  // the row fits in one workgroup's registers
    if (s.kprec)
      k_cg32_alpha_row<true, kAlphaMaxPer><<<n, kAlphaThreads, 0, st>>>(s, act, tol2, live);
    else
      k_cg32_alpha_row<false, kAlphaMaxPer><<<n, kAlphaThreads, 0, st>>>(s, act, tol2, live);
  } else if (s.kprec) {
    k_cg32_alpha<true><<<n, kCgThreads, 0, st>>>(s, act, tol2, live);
  } else {
    k_cg32_alpha<false><<<n, kCgThreads, 0, st>>>(s, act, tol2, live);
  }
}

// In-place stable compaction of the active list by one workgroup of 1024 threads:
// chunk by chunk, every entry of a chunk is read before any is written, and an
// entry moves to its position among the kept ones, at or before where it was
// read, so nothing is overwritten before it is read. The count is read by every
// thread at the start and written by thread 0 after the last barrier.
constexpr int kCompactThreads = 1024;
__global__ __launch_bounds__(kCompactThreads) void k_compact(int* __restrict__ list, int* __restrict__ count,
                                                             const int* __restrict__ flag) {
  __shared__ int wsum[kCompactThreads / 64];
  const int n = *count;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int base = 0;  // kept entries before the current chunk (the same in every thread)
  for (int c0 = 0; c0 < n; c0 += kCompactThreads) {
    const int i = c0 + threadIdx.x;
    int s = 0, keep = 0;
    if (i < n) {
      s = list[i];
      keep = flag[s] == 0;
    }
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();  // every read of this chunk is done; the wave sums are visible
    int off = base, tot = 0;
#pragma unroll
    for (int w = 0; w < kCompactThreads / 64; ++w) {
      off += w < wave ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (keep) list[off + before] = s;
    base += tot;
    __syncthreads();  // wsum is reused by the next chunk
  }
  if (threadIdx.x == 0) *count = base;
}

void launch_compact(int* list, int* count, const int* flag, hipStream_t st) {
  k_compact<<<1, kCompactThreads, 0, st>>>(list, count, flag);
}
void launch_cg32_beta(const Cg32State& s, const int* act, int n, hipStream_t st, const int* live) {
  if (n > 0) k_cg32_beta<<<n, kCgThreads, 0, st>>>(s, act, live);
}
__global__ void k_set_int(int* __restrict__ p, int v) { *p = v; }
void launch_set_int(int* p, int v, hipStream_t st) { k_set_int<<<1, 1, 0, st>>>(p, v); }
void launch_add_d(Z64* x, const Z32* d, int ld, const int* act, int n, hipStream_t st) {
  if (n > 0) k_add_d<<<n, 256, 0, st>>>(x, d, ld, act);
}
void launch_outer_resid(const CgState& s, const int* act, int n, double tol, hipStream_t st) {
  if (n > 0) k_outer_resid<<<n, kCgThreads, 0, st>>>(s, act, tol);
}
void launch_row_norm2(const Z64* y, int ld, int n, double* out, hipStream_t st) {
  if (n > 0) k_row_norm2<<<n, kCgThreads, 0, st>>>(y, ld, out);
}
void launch_outer_init(const CgState& s, const int* act, int n, double cut, hipStream_t st) {
  if (n > 0) k_outer_init<<<n, kCgThreads, 0, st>>>(s, act, cut * cut);
}
void launch_fill_zero32(Z32* p, size_t n, hipStream_t st) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fill_zero32<<<(unsigned)blocks, 256, 0, st>>>(p, n);
}
void launch_row_dot(const Z64* a, const Z64* b, int ld, int nrows, Z64* out, hipStream_t st) {
  if (nrows > 0) k_row_dot<<<nrows, kCgThreads, 0, st>>>(a, b, ld, out);
}
void launch_blk_axpy(Z64* y, const Z64* x, const Z64* c, int nb, int ld, int nrows, hipStream_t st) {
  if (nrows > 0) k_blk_axpy<<<nrows, kCgThreads, 0, st>>>(y, x, c, nb, ld);
}
void launch_blk_xpby(Z64* p, const Z64* z, const Z64* c, int nb, int ld, int nrows, hipStream_t st) {
  if (nrows > 0) k_blk_xpby<<<nrows, kCgThreads, 0, st>>>(p, z, c, nb, ld);
}
void launch_blk_scale(Z64* y, const Z64* c, int nb, int ld, int nrows, hipStream_t st) {
  if (nrows > 0) k_blk_scale<<<nrows, kCgThreads, 0, st>>>(y, c, nb, ld);
}
void launch_teter_rows(const Z64* r, Z64* z, const double* g2h, const double* invT, int nb, int ld, int nrows,
                       hipStream_t st) {
  if (nrows > 0) k_teter_rows<<<nrows, kCgThreads, 0, st>>>(r, z, g2h, invT, nb, ld);
}

}  // namespace stern
