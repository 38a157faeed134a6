// Complex GEMMs of the mixed-precision inner solve on the gfx950 BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// Every operand is carried as a split pair hi + lo of BF16 numbers
// (hi = bf16(v), lo = bf16(v - hi)), and each product is formed as
// hi*hi + hi*lo + lo*hi, which keeps about 16 significant bits. Psi and the KB
// rows are split once (set_occupied / init); the FP32 vectors are split in
// registers while they are loaded. Complex arithmetic uses the interleaved
// real layout (re, im, re, im, ...) along the reduction index:
//   Re conj(a) x = (a_re, a_im) . (x_re, x_im),  Im conj(a) x = (a_re, a_im) . (x_im, -x_re)
//   Re a c       = (a_re, a_im) . (c_re, -c_im), Im a c       = (a_re, a_im) . (c_im, c_re)
// so no lane ever needs another lane's data.
#include "kernels.hpp"

namespace stern {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// split 8 floats into bf16 hi and lo parts
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)v[e];
    hi[e] = h;
    lo[e] = (__bf16)(v[e] - (float)h);
  }
}

constexpr int kThreads = 256;  // 4 waves in a 2 x 2 arrangement of 32 x 32 tiles

// C[n][m] partial over this split's K range = sum_k conj(A[m][k]) X[xidx[n]][k]
// A: hi/lo [M_pad][2 K] bf16 interleaved; X: [rows][ldx] complex float
__global__ __launch_bounds__(kThreads) void k_reduce_bf16(const __bf16* __restrict__ Ahi,
                                                          const __bf16* __restrict__ Alo, int M_pad,
                                                          const Z32* __restrict__ X, int ldx,
                                                          const int* __restrict__ xidx, int ncols, int K,
                                                          int kchunk, Z32* __restrict__ cpart) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int split = blockIdx.z;
  const int kb = split * kchunk;
  const int ke = min(K, kb + kchunk);
  const __bf16* ah[2];
  const __bf16* al[2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const size_t row = (size_t)(m0 + 16 * bi + l16) * 2 * K;
    ah[bi] = Ahi + row;
    al[bi] = Alo + row;
  }
  const Z32* xr[2];
  bool xv[2];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int n = n0 + 16 * bj + l16;
    xv[bj] = n < ncols;
    xr[bj] = X + (size_t)(xv[bj] ? (xidx ? xidx[n] : n) : 0) * ldx;
  }
  f32x4 cre[2][2], cim[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      cre[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  for (int kc = kb; kc < ke; kc += 16) {
    const int k = kc + 4 * g;  // this lane group's 4 complex k
    bf16x8 a_hi[2], a_lo[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      a_hi[bi] = *reinterpret_cast<const bf16x8*>(ah[bi] + 2 * k);
      a_lo[bi] = *reinterpret_cast<const bf16x8*>(al[bi] + 2 * k);
    }
    bf16x8 xr_hi[2], xr_lo[2], xi_hi[2], xi_lo[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      float re8[8], im8[8];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        Z32 v = zmk(0.f, 0.f);
        if (xv[bj]) v = xr[bj][k + t];
        re8[2 * t] = v.re;
        re8[2 * t + 1] = v.im;
        im8[2 * t] = v.im;
        im8[2 * t + 1] = -v.re;
      }
      split8(re8, xr_hi[bj], xr_lo[bj]);
      split8(im8, xi_hi[bj], xi_lo[bj]);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        cre[bi][bj] = mfma(a_hi[bi], xr_hi[bj], cre[bi][bj]);
        cre[bi][bj] = mfma(a_hi[bi], xr_lo[bj], cre[bi][bj]);
        cre[bi][bj] = mfma(a_lo[bi], xr_hi[bj], cre[bi][bj]);
        cim[bi][bj] = mfma(a_hi[bi], xi_hi[bj], cim[bi][bj]);
        cim[bi][bj] = mfma(a_hi[bi], xi_lo[bj], cim[bi][bj]);
        cim[bi][bj] = mfma(a_lo[bi], xi_hi[bj], cim[bi][bj]);
      }
  }
  // D[i][j]: column j = lane % 16, row i = 4 (lane / 16) + r
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int n = n0 + 16 * bj + l16;
    if (n >= ncols) continue;
    Z32* dst = cpart + ((size_t)split * ncols + n) * M_pad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[m0 + 16 * bi + 4 * g + r] = zmk(cre[bi][bj][r], cim[bi][bj][r]);
  }
}

__global__ void k_sum_parts32(const Z32* __restrict__ cpart, int nsplit, int total, float scale, Z32* __restrict__ C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float re = 0.f, im = 0.f;
  for (int s = 0; s < nsplit; ++s) {
    const Z32 v = cpart[(size_t)s * total + i];
    re += v.re;
    im += v.im;
  }
  C[i] = zmk(scale * re, scale * im);
}

// Y[yidx[n]][k] += sum_m A[m][k] C[n][m]; AT: hi/lo [K][2 M_pad] bf16 interleaved along m
__global__ __launch_bounds__(kThreads) void k_expand_bf16(const __bf16* __restrict__ ATh,
                                                          const __bf16* __restrict__ ATl, int M_pad, int K,
                                                          const Z32* __restrict__ C, Z32* __restrict__ Y, int ldy,
                                                          const int* __restrict__ yidx, int ncols) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int k0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
  int nn[2];
  bool nv[2];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    nn[bj] = n0 + 16 * bj + l16;
    nv[bj] = nn[bj] < ncols;
  }
  f32x4 dre[2][2], dim_[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      dre[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
      dim_[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  for (int mc = 0; mc < M_pad; mc += 16) {
    const int m = mc + 4 * g;  // this lane group's 4 complex m
    bf16x8 a_hi[2], a_lo[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const size_t row = (size_t)(k0 + 16 * bi + l16) * 2 * M_pad + 2 * m;
      a_hi[bi] = *reinterpret_cast<const bf16x8*>(ATh + row);
      a_lo[bi] = *reinterpret_cast<const bf16x8*>(ATl + row);
    }
    bf16x8 cr_hi[2], cr_lo[2], ci_hi[2], ci_lo[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      float re8[8], im8[8];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        Z32 c = zmk(0.f, 0.f);
        if (nv[bj]) c = C[(size_t)nn[bj] * M_pad + m + t];
        re8[2 * t] = c.re;
        re8[2 * t + 1] = -c.im;
        im8[2 * t] = c.im;
        im8[2 * t + 1] = c.re;
      }
      split8(re8, cr_hi[bj], cr_lo[bj]);
      split8(im8, ci_hi[bj], ci_lo[bj]);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        dre[bi][bj] = mfma(a_hi[bi], cr_hi[bj], dre[bi][bj]);
        dre[bi][bj] = mfma(a_hi[bi], cr_lo[bj], dre[bi][bj]);
        dre[bi][bj] = mfma(a_lo[bi], cr_hi[bj], dre[bi][bj]);
        dim_[bi][bj] = mfma(a_hi[bi], ci_hi[bj], dim_[bi][bj]);
        dim_[bi][bj] = mfma(a_hi[bi], ci_lo[bj], dim_[bi][bj]);
        dim_[bi][bj] = mfma(a_lo[bi], ci_hi[bj], dim_[bi][bj]);
      }
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    if (!nv[bj]) continue;
    Z32* y = Y + (size_t)(yidx ? yidx[nn[bj]] : nn[bj]) * ldy;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + 16 * bi + 4 * g + r;
        const Z32 old = y[k];
        y[k] = zmk(old.re + dre[bi][bj][r], old.im + dim_[bi][bj][r]);
      }
  }
}

// hi/lo split of complex double rows [M][K] into row layout [M][2K] and the
// transposed layout [K][2 M] (both interleaved re, im)
__global__ void k_split_rows(const Z64* __restrict__ A, int M, int K, __bf16* __restrict__ hi, __bf16* __restrict__ lo,
                             __bf16* __restrict__ thi, __bf16* __restrict__ tlo) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)M * K) return;
  const int m = (int)(i / K), k = (int)(i - (size_t)m * K);
  const Z64 v = A[i];
  const float re = (float)v.re, im = (float)v.im;
  const __bf16 hr = (__bf16)re, hm = (__bf16)im;
  const __bf16 lr = (__bf16)(float)(v.re - (double)(float)hr);
  const __bf16 lm = (__bf16)(float)(v.im - (double)(float)hm);
  hi[2 * i] = hr;
  hi[2 * i + 1] = hm;
  lo[2 * i] = lr;
  lo[2 * i + 1] = lm;
  const size_t t = (size_t)k * 2 * M + 2 * m;
  thi[t] = hr;
  thi[t + 1] = hm;
  tlo[t] = lr;
  tlo[t + 1] = lm;
}

}  // namespace

int choose_nsplit_bf16(int M_pad, int ncols, int K) {
  const int base = (M_pad / 64) * ((ncols + 63) / 64);
  int ns = (2048 + base - 1) / base;
  const int maxs = K / 512 > 0 ? K / 512 : 1;
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return ns;
}

void launch_split_bf16(const Z64* A, int M, int K, __bf16* hi, __bf16* lo, __bf16* thi, __bf16* tlo, hipStream_t st) {
  const size_t n = (size_t)M * K;
  if (n == 0) return;
  k_split_rows<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(A, M, K, hi, lo, thi, tlo);
}

void launch_reduce_bf16(const __bf16* Ahi, const __bf16* Alo, int M_pad, const Z32* X, int ldx, const int* xidx,
                        int ncols, int K, Z32* cpart, int nsplit, hipStream_t st) {
  if (ncols <= 0) return;
  int kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 15) / 16 * 16;
  dim3 grid(M_pad / 64, (ncols + 63) / 64, nsplit);
  k_reduce_bf16<<<grid, kThreads, 0, st>>>(Ahi, Alo, M_pad, X, ldx, xidx, ncols, K, kchunk, cpart);
}

void launch_sum_parts32(const Z32* cpart, int nsplit, int ncols, int M_pad, float scale, Z32* C, hipStream_t st) {
  const int total = ncols * M_pad;
  if (total <= 0) return;
  k_sum_parts32<<<(total + 255) / 256, 256, 0, st>>>(cpart, nsplit, total, scale, C);
}

void launch_expand_bf16(const __bf16* ATh, const __bf16* ATl, int M_pad, const Z32* C, Z32* Y, int ldy,
                        const int* yidx, int ncols, int K, hipStream_t st) {
  if (ncols <= 0) return;
  dim3 grid(K / 64, (ncols + 63) / 64);
  k_expand_bf16<<<grid, kThreads, 0, st>>>(ATh, ATl, M_pad, K, C, Y, ldy, yidx, ncols);
}

}  // namespace stern
