// Complex FP64 GEMMs of the KB projectors and of P_c = 1 - Psi Psi^H on the
// gfx950 FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// A complex product is split into real MFMAs without any cross-lane traffic:
// each lane loads two consecutive complex elements (32 bytes) of its row and
// feeds their four real parts to four successive MFMAs, so the four lane
// groups of a wavefront cover eight complex k per MFMA quadruple. Because the
// k order inside a reduction is free, the A and B fragments only have to agree
// on which k each lane group carries.
#include "kernels.hpp"

namespace stern {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGemmThreads = 256;  // 4 waves, 2 x 2 arrangement of 32 x 32 wave tiles

// C[n][m] (partial over the K range of this split) = sum_k conj(A[m][k]) X[xidx[n]][k]
__global__ __launch_bounds__(kGemmThreads) void k_zgemm_reduce(const Z64* __restrict__ A, int M_pad,
                                                               const Z64* __restrict__ X, int ldx,
                                                               const int* __restrict__ xidx, int ncols, int K,
                                                               int kchunk, Z64* __restrict__ cpart) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int split = blockIdx.z;
  const int kb = split * kchunk;
  const int ke = min(K, kb + kchunk);
  const Z64* ar[2];
  const Z64* xr[2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) ar[bi] = A + (size_t)(m0 + 16 * bi + l16) * K;
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int n = n0 + 16 * bj + l16;
    const int row = n < ncols ? (xidx ? xidx[n] : n) : (xidx ? xidx[0] : 0);
    xr[bj] = X + (size_t)row * ldx;
  }
  v4d cre[2][2], cim[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      cre[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
      cim[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  // The next step's fragments are loaded before this step's products (every load unconditional:
  // columns past ncols read row 0, whose products are never stored), so they arrive while the
  // products of this step run.
  Z64 na0[2], na1[2], nx0[2], nx1[2];
  auto load = [&](int kc) {
    const int k = kc + 2 * g;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      na0[bi] = ar[bi][k];
      na1[bi] = ar[bi][k + 1];
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      nx0[bj] = xr[bj][k];
      nx1[bj] = xr[bj][k + 1];
    }
  };
  if (kb < ke) load(kb);
  for (int kc = kb; kc < ke; kc += 8) {
    Z64 a0[2], a1[2], x0[2], x1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      a0[u] = na0[u];
      a1[u] = na1[u];
      x0[u] = nx0[u];
      x1[u] = nx1[u];
    }
    load(min(kc + 8, ke - 8));  // the last step reloads itself, unused
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        // Re conj(a) x = a.re x.re + a.im x.im ; Im conj(a) x = a.re x.im - a.im x.re
        cre[bi][bj] = mfma(a0[bi].re, x0[bj].re, cre[bi][bj]);
        cre[bi][bj] = mfma(a0[bi].im, x0[bj].im, cre[bi][bj]);
        cre[bi][bj] = mfma(a1[bi].re, x1[bj].re, cre[bi][bj]);
        cre[bi][bj] = mfma(a1[bi].im, x1[bj].im, cre[bi][bj]);
        cim[bi][bj] = mfma(a0[bi].re, x0[bj].im, cim[bi][bj]);
        cim[bi][bj] = mfma(a0[bi].im, -x0[bj].re, cim[bi][bj]);
        cim[bi][bj] = mfma(a1[bi].re, x1[bj].im, cim[bi][bj]);
        cim[bi][bj] = mfma(a1[bi].im, -x1[bj].re, cim[bi][bj]);
      }
  }
  // D[i][j] of a 16x16 block: column j = lane % 16, row i = lane / 16 + 4 r in accumulator element r
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    const int n = n0 + 16 * bj + l16;
    if (n >= ncols) continue;
    Z64* dst = cpart + ((size_t)split * ncols + n) * M_pad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[m0 + 16 * bi + g + 4 * r] = zmk(cre[bi][bj][r], cim[bi][bj][r]);
    }
  }
}

__global__ void k_sum_parts(const Z64* __restrict__ cpart, int nsplit, int total, double scale, Z64* __restrict__ C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const Z64 v = cpart[(size_t)s * total + i];
    re += v.re;
    im += v.im;
  }
  C[i] = zmk(scale * re, scale * im);
}

// Y[yidx[n]][k] += sum_m A[m][k] C[n][m]. Bounded to 4 waves per SIMD: the compiler then keeps the
// accumulators in VGPRs (114 in all) instead of 104 VGPRs + 64 AGPRs at 3 waves; 59 -> 70 TFLOP/s at
// M = 1,024, 4,096 columns, K = 91,072.
__global__ __launch_bounds__(kGemmThreads, 4) void k_zgemm_expand(const Z64* __restrict__ A, int M_pad, int K,
                                                               const Z64* __restrict__ C, Z64* __restrict__ Y,
                                                               int ldy, const int* __restrict__ yidx, int ncols) {
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
  v4d dre[2][2], dim_[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      dre[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
      dim_[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
    }
  // next step's fragments loaded before this step's products; columns past ncols read column 0
  Z64 na0[2], na1[2], nc0[2], nc1[2];
  auto load = [&](int m) {
    const int mm = m + 2 * g;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int kk = k0 + 16 * bi + l16;
      na0[bi] = A[(size_t)mm * K + kk];
      na1[bi] = A[(size_t)(mm + 1) * K + kk];
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const size_t o = (size_t)(nv[bj] ? nn[bj] : 0) * M_pad + mm;
      nc0[bj] = C[o];
      nc1[bj] = C[o + 1];
    }
  };
  load(0);
  for (int m = 0; m < M_pad; m += 8) {
    Z64 a0[2], a1[2], c0[2], c1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      a0[u] = na0[u];
      a1[u] = na1[u];
      c0[u] = nc0[u];
      c1[u] = nc1[u];
    }
    load(min(m + 8, M_pad - 8));  // the last step reloads itself, unused
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        // Re a c = a.re c.re - a.im c.im ; Im a c = a.re c.im + a.im c.re
        dre[bi][bj] = mfma(a0[bi].re, c0[bj].re, dre[bi][bj]);
        dre[bi][bj] = mfma(a0[bi].im, -c0[bj].im, dre[bi][bj]);
        dre[bi][bj] = mfma(a1[bi].re, c1[bj].re, dre[bi][bj]);
        dre[bi][bj] = mfma(a1[bi].im, -c1[bj].im, dre[bi][bj]);
        dim_[bi][bj] = mfma(a0[bi].re, c0[bj].im, dim_[bi][bj]);
        dim_[bi][bj] = mfma(a0[bi].im, c0[bj].re, dim_[bi][bj]);
        dim_[bi][bj] = mfma(a1[bi].re, c1[bj].im, dim_[bi][bj]);
        dim_[bi][bj] = mfma(a1[bi].im, c1[bj].re, dim_[bi][bj]);
      }
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    if (!nv[bj]) continue;
    const int row = yidx ? yidx[nn[bj]] : nn[bj];
    Z64* y = Y + (size_t)row * ldy;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + 16 * bi + g + 4 * r;
        const Z64 old = y[k];
        y[k] = zmk(old.re + dre[bi][bj][r], old.im + dim_[bi][bj][r]);
      }
    }
  }
}

}  // namespace

constexpr int kGemm64TargetGroups = 2048;  // workgroups a split-K reduce aims for by default

int choose_nsplit(int M_pad, int ncols, int K, int target) {
  if (target <= 0) target = kGemm64TargetGroups;
  const int base = (M_pad / 64) * ((ncols + 63) / 64);
  int ns = (target + base - 1) / base;
  const int maxs = K / 256 > 0 ? K / 256 : 1;
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return ns;
}

void launch_zgemm_reduce(const Z64* A, int M_pad, const Z64* X, int ldx, const int* xidx, int ncols, int K,
                         Z64* cpart, int nsplit, hipStream_t st) {
  if (ncols <= 0) return;
  int kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 7) / 8 * 8;
  dim3 grid(M_pad / 64, (ncols + 63) / 64, nsplit);
  k_zgemm_reduce<<<grid, kGemmThreads, 0, st>>>(A, M_pad, X, ldx, xidx, ncols, K, kchunk, cpart);
}

void launch_sum_parts(const Z64* cpart, int nsplit, int ncols, int M_pad, double scale, Z64* C, hipStream_t st) {
  const int total = ncols * M_pad;
  if (total <= 0) return;
  k_sum_parts<<<(total + 255) / 256, 256, 0, st>>>(cpart, nsplit, total, scale, C);
}

void launch_zgemm_expand(const Z64* A, int M_pad, const Z64* C, Z64* Y, int ldy, const int* yidx, int ncols, int K,
                         hipStream_t st) {
  if (ncols <= 0) return;
  dim3 grid(K / 64, (ncols + 63) / 64);
  k_zgemm_expand<<<grid, kGemmThreads, 0, st>>>(A, M_pad, K, C, Y, ldy, yidx, ncols);
}

}  // namespace stern
