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
#include <utility>

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

constexpr int kThreads = 256;  // 4 waves
constexpr int kBf16TargetGroups = 512;  // workgroups a split-K reduce aims for

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// (-a_im, a_re) for each complex (a_re, a_im) of an interleaved bf16x8: rotate
// every dword by 16 bits and flip the sign of the new low half
__device__ __forceinline__ bf16x8 rot_neg(bf16x8 a) {
  u32x4 d = __builtin_bit_cast(u32x4, a);
#pragma unroll
  for (int e = 0; e < 4; ++e) d[e] = __builtin_amdgcn_alignbit(d[e], d[e], 16) ^ 0x8000u;
  return __builtin_bit_cast(bf16x8, d);
}

// 4 complex floats (interleaved re, im) -> bf16 hi and lo
__device__ __forceinline__ void split_z4(const Z32 (&v)[4], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const __bf16 hr = (__bf16)v[t].re, hm = (__bf16)v[t].im;
    hi[2 * t] = hr;
    hi[2 * t + 1] = hm;
    lo[2 * t] = (__bf16)(v[t].re - (float)hr);
    lo[2 * t + 1] = (__bf16)(v[t].im - (float)hm);
  }
}

constexpr int kWM = 128;     // reduce: rows of A per workgroup (4 row groups of 32)
constexpr int kWN = 128;     // reduce: columns per workgroup (2 column groups of 64)
constexpr int kET = 256;     // expand: rows k per workgroup (4 groups of 64)
constexpr int kEN = 128;     // expand: columns per workgroup (2 groups of 64)
constexpr int kThreads8 = 512;

// C[n][m] partial over this split's K range = sum_k conj(A[m][k]) X[xidx[n]][k].
// 8 waves: wave (wm, wn) owns rows [32 wm, 32 wm + 32) and columns
// [64 wn, 64 wn + 64) of the 128 x 128 tile. A K step covers 32 complex, two MFMA
// sub-steps of 16: the 128 x 32 slice of X is split into bf16 hi/lo once and staged
// in LDS (double-buffered, [sub-step][column][group of 4 complex]); A's fragments of
// the next step are loaded while this step's MFMAs run. Re C = A . X and
// Im C = A' . X along the interleaved reduction index, with A' = (-a_im, a_re)
// formed from A in registers.
// Workgroups are numbered so that the row blocks of one (column block, split)
// pair get consecutive slots of one XCD (the hardware hands workgroup L to XCD
// L mod 8): they run together and share that pair's slice of X through the
// XCD's L2 instead of each fetching it from HBM.
__global__ __launch_bounds__(kThreads8) void k_reduce_bf16w(const __bf16* __restrict__ Ahi,
                                                            const __bf16* __restrict__ Alo, int M_pad,
                                                            const Z32* __restrict__ X, int ldx,
                                                            const int* __restrict__ xidx, int ncols, int K,
                                                            int kchunk, Z32* __restrict__ cpart, int nmb, int nnb,
                                                            int nsplit, const int* __restrict__ ncount) {
  __shared__ bf16x8 xs[2][2][2][kWN * 4];  // [buffer][hi, lo][sub-step][column * 4 + group of 4 complex]
  const int L = blockIdx.x, slot = L >> 3;
  const int mb = slot % nmb, rest = (slot / nmb) * 8 + (L & 7);
  if (rest >= nnb * nsplit) return;  // padding of the last group of XCD slots; no barrier passed yet
  const int nlive = ncount ? min(ncols, *ncount) : ncols;  // ncols stays the stride of the partials
  if ((rest % nnb) * kWN >= nlive) return;  // no live column in this block; no barrier passed yet
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int wm = wave & 3, wn = wave >> 2;
  const int n0 = (rest % nnb) * kWN;
  const int split = rest / nnb;
  const int m0 = mb * kWM + wm * 32;
  const bool live = m0 < M_pad;
  const int kb = split * kchunk;
  const int ke = min(K, kb + kchunk);
  // staging: thread -> (column tn, 8 complex from 8 tq): groups 2 tq and 2 tq + 1 of the step
  const int tn = threadIdx.x >> 2, tq = threadIdx.x & 3;
  const int ncol = n0 + tn;
  const bool xval = ncol < nlive;
  const Z32* xrow = X + (size_t)(xval ? (xidx ? xidx[ncol] : ncol) : 0) * ldx;
  const __bf16* ah[2];
  const __bf16* al[2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const size_t row = (size_t)(live ? m0 + 16 * bi + l16 : 0) * 2 * K;
    ah[bi] = Ahi + row;
    al[bi] = Alo + row;
  }
  f32x4 cre[2][4], cim[2][4];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      cre[bi][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[bi][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  Z32 xv[8];
  auto load_x = [&](int kc) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      xv[t] = zmk(0.f, 0.f);
      if (xval) xv[t] = xrow[kc + 8 * tq + t];
    }
  };
  auto put_x = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int G = 2 * tq + h;  // group of 4 complex within the step
      bf16x8 hi, lo;
      split_z4(*reinterpret_cast<const Z32(*)[4]>(xv + 4 * h), hi, lo);
      xs[buf][0][G >> 2][tn * 4 + (G & 3)] = hi;
      xs[buf][1][G >> 2][tn * 4 + (G & 3)] = lo;
    }
  };
  bf16x8 a_hi[2][2], a_lo[2][2];
  auto load_a = [&](int kc) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int k = kc + 16 * kk + 4 * g;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        a_hi[kk][bi] = *reinterpret_cast<const bf16x8*>(ah[bi] + 2 * k);
        a_lo[kk][bi] = *reinterpret_cast<const bf16x8*>(al[bi] + 2 * k);
      }
    }
  };
  if (kb < ke) {
    load_x(kb);
    put_x(0);
    if (live) load_a(kb);
  }
  __syncthreads();
  int buf = 0;
  for (int kc = kb; kc < ke; kc += 32) {
    const bool more = kc + 32 < ke;
    if (more) load_x(kc + 32);  // in flight during the MFMAs
    if (live) {
      bf16x8 c_hi[2][2], c_lo[2][2], b_hi[2][2], b_lo[2][2];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
          c_hi[kk][bi] = a_hi[kk][bi];
          c_lo[kk][bi] = a_lo[kk][bi];
          b_hi[kk][bi] = rot_neg(c_hi[kk][bi]);
          b_lo[kk][bi] = rot_neg(c_lo[kk][bi]);
        }
      if (more) load_a(kc + 32);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int col = wn * 64 + nb * 16 + l16;
          const bf16x8 x_hi = xs[buf][0][kk][col * 4 + g];
          const bf16x8 x_lo = xs[buf][1][kk][col * 4 + g];
#pragma unroll
          for (int bi = 0; bi < 2; ++bi) {
            cre[bi][nb] = mfma(c_hi[kk][bi], x_hi, cre[bi][nb]);
            cre[bi][nb] = mfma(c_hi[kk][bi], x_lo, cre[bi][nb]);
            cre[bi][nb] = mfma(c_lo[kk][bi], x_hi, cre[bi][nb]);
            cim[bi][nb] = mfma(b_hi[kk][bi], x_hi, cim[bi][nb]);
            cim[bi][nb] = mfma(b_hi[kk][bi], x_lo, cim[bi][nb]);
            cim[bi][nb] = mfma(b_lo[kk][bi], x_hi, cim[bi][nb]);
          }
        }
    }
    if (more) put_x(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (!live) return;
  // D[i][j]: column j = lane % 16 (vector), row i = 4 (lane / 16) + r
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int n = n0 + wn * 64 + nb * 16 + l16;
    if (n >= nlive) continue;
    Z32* dst = cpart + ((size_t)split * ncols + n) * M_pad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[m0 + 16 * bi + 4 * g + r] = zmk(cre[bi][nb][r], cim[bi][nb][r]);
  }
}

// C = scale * sum of the split partials, as bf16 hi and lo of (c_re, c_im):
// Cs[0], Cs[1], each [ncols][2 M_pad] interleaved along m.
__global__ void k_sum_split(const Z32* __restrict__ cpart, int nsplit, int ncols, int M_pad, float scale,
                            __bf16* __restrict__ Cs, const int* __restrict__ live) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = ncols * M_pad;
  if (i >= total || (live && i / M_pad >= *live)) return;
  float re = 0.f, im = 0.f;
  for (int s = 0; s < nsplit; ++s) {
    const Z32 v = cpart[(size_t)s * total + i];
    re += v.re;
    im += v.im;
  }
  re *= scale;
  im *= scale;
  const size_t plane = (size_t)total * 2;
  const __bf16 rh = (__bf16)re, ih = (__bf16)im;
  Cs[2 * (size_t)i] = rh;
  Cs[2 * (size_t)i + 1] = ih;
  Cs[plane + 2 * (size_t)i] = (__bf16)(re - (float)rh);
  Cs[plane + 2 * (size_t)i + 1] = (__bf16)(im - (float)ih);
}

// (c_re, -c_im) and (c_im, c_re) of an interleaved bf16x8 of (c_re, c_im)
__device__ __forceinline__ bf16x8 conj_b(bf16x8 c) {
  u32x4 d = __builtin_bit_cast(u32x4, c);
#pragma unroll
  for (int e = 0; e < 4; ++e) d[e] ^= 0x80000000u;
  return __builtin_bit_cast(bf16x8, d);
}
__device__ __forceinline__ bf16x8 swap_b(bf16x8 c) {
  u32x4 d = __builtin_bit_cast(u32x4, c);
#pragma unroll
  for (int e = 0; e < 4; ++e) d[e] = __builtin_amdgcn_alignbit(d[e], d[e], 16);
  return __builtin_bit_cast(bf16x8, d);
}

// Y[yidx[n]][k] += sum_m A[m][k] C[n][m], A given transposed (AT [K][2 M_pad]
// hi/lo) and C as k_sum_split writes it. PUPD: Y is left as it is and the sum
// goes into the search direction instead, P[s] = (Y[s] + A C) + beta[s] P[s]
// (s = yidx[n]), the CG direction update from the projected z. 4 WN waves: wave (wk, wn) owns
// rows [16 KB wk, 16 KB (wk + 1)) and columns [64 wn, 64 wn + 64) of the
// (64 KB) x (64 WN) tile: KB = 4, WN = 2 (256 x 128, 1 workgroup per CU); KB = 2, WN = 2
// (128 x 128, fewer registers, 2 workgroups per CU); KB = 4, WN = 1 (256 x 64, 2 workgroups
// per CU). With two workgroups on a CU one's Y update overlaps the other's products.
// Re(a c) = a . (c_re, -c_im), Im(a c) = a . (c_im, c_re).
// Workgroups are numbered so that the column blocks of one row block k get
// consecutive slots of one XCD (workgroup L runs on XCD L mod 8) and share
// that block's rows of A through the XCD's L2.
template <int KB, bool PUPD, int WN>
__global__ __launch_bounds__(256 * WN, KB == 4 ? 2 : 4) void k_expand_bf16s(const __bf16* __restrict__ ATh,
                                                            const __bf16* __restrict__ ATl, int M_pad, int K,
                                                            const __bf16* __restrict__ Cs, Z32* __restrict__ Y,
                                                            int ldy, const int* __restrict__ yidx, int ncols,
                                                            Z32* __restrict__ P, const double* __restrict__ beta,
                                                            int nnb, const int* __restrict__ live) {
  const int nlive = live ? min(ncols, *live) : ncols;  // ncols stays the stride of C
  const int L = blockIdx.x, slot = L >> 3;
  const int nbk = slot % nnb, kblk = (slot / nnb) * 8 + (L & 7);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int wk = wave & 3, wn = wave >> 2;
  const int k0 = kblk * (64 * KB) + wk * 16 * KB;
  if (k0 >= K) return;  // K is a multiple of 64; no barrier below
  const int n0 = nbk * (64 * WN) + wn * 64;
  if (n0 >= nlive) return;  // no live column for this wave
  const size_t plane = (size_t)ncols * M_pad * 2;
  int nn[4];
  bool nv[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    nn[bj] = n0 + 16 * bj + l16;
    nv[bj] = nn[bj] < nlive;
  }
  f32x4 dre[KB][4], dim_[KB][4];
#pragma unroll
  for (int bi = 0; bi < KB; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      dre[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
      dim_[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  const bf16x8 zero8 = bf16x8{};
  for (int mc = 0; mc < M_pad; mc += 16) {
    const int m = mc + 4 * g;  // this lane group's 4 complex m
    bf16x8 a_hi[KB], a_lo[KB];
#pragma unroll
    for (int bi = 0; bi < KB; ++bi) {
      const size_t row = (size_t)(k0 + 16 * bi + l16) * 2 * M_pad + 2 * m;
      a_hi[bi] = *reinterpret_cast<const bf16x8*>(ATh + row);
      a_lo[bi] = *reinterpret_cast<const bf16x8*>(ATl + row);
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      bf16x8 ch = zero8, cl = zero8;
      if (nv[bj]) {
        const size_t o = (size_t)nn[bj] * 2 * M_pad + 2 * m;
        ch = *reinterpret_cast<const bf16x8*>(Cs + o);
        cl = *reinterpret_cast<const bf16x8*>(Cs + plane + o);
      }
      const bf16x8 rh = conj_b(ch), rl = conj_b(cl), ih = swap_b(ch), il = swap_b(cl);
#pragma unroll
      for (int bi = 0; bi < KB; ++bi) {
        dre[bi][bj] = mfma(a_hi[bi], rh, dre[bi][bj]);
        dre[bi][bj] = mfma(a_hi[bi], rl, dre[bi][bj]);
        dre[bi][bj] = mfma(a_lo[bi], rh, dre[bi][bj]);
        dim_[bi][bj] = mfma(a_hi[bi], ih, dim_[bi][bj]);
        dim_[bi][bj] = mfma(a_hi[bi], il, dim_[bi][bj]);
        dim_[bi][bj] = mfma(a_lo[bi], ih, dim_[bi][bj]);
      }
    }
  }
  // D[i][j]: column j = lane % 16 (vector), rows i = 4 (lane / 16) + r: 4 consecutive k per lane
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    if (!nv[bj]) continue;
    const size_t row = (size_t)(yidx ? yidx[nn[bj]] : nn[bj]);
    Z32* y = Y + row * ldy;
    float bt = 0.f;
    if constexpr (PUPD) bt = (float)beta[row];
#pragma unroll
    for (int bi = 0; bi < KB; ++bi) {
      float4* p = reinterpret_cast<float4*>(y + k0 + 16 * bi + 4 * g);
      float4 u = p[0], w = p[1];
      u.x += dre[bi][bj][0];
      u.y += dim_[bi][bj][0];
      u.z += dre[bi][bj][1];
      u.w += dim_[bi][bj][1];
      w.x += dre[bi][bj][2];
      w.y += dim_[bi][bj][2];
      w.z += dre[bi][bj][3];
      w.w += dim_[bi][bj][3];
      if constexpr (PUPD) {
        float4* d = reinterpret_cast<float4*>(P + row * ldy + k0 + 16 * bi + 4 * g);
        const float4 a = d[0], c = d[1];
        d[0] = make_float4(u.x + bt * a.x, u.y + bt * a.y, u.z + bt * a.z, u.w + bt * a.w);
        d[1] = make_float4(w.x + bt * c.x, w.y + bt * c.y, w.z + bt * c.z, w.w + bt * c.w);
      } else {
        p[0] = u;
        p[1] = w;
      }
    }
  }
}

// hi/lo split of complex double rows [M][K] into rows [row0, row0 + M) of a
// matrix of Mt rows, in row layout [Mt][2K] (skipped when hi is null) and
// transposed layout [K][2 Mt] (both interleaved re, im)
__global__ void k_split_rows(const Z64* __restrict__ A, int M, int K, int row0, int Mt, __bf16* __restrict__ hi,
                             __bf16* __restrict__ lo, __bf16* __restrict__ thi, __bf16* __restrict__ tlo) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)M * K) return;
  const int m = (int)(i / K), k = (int)(i - (size_t)m * K);
  const Z64 v = A[i];
  const float re = (float)v.re, im = (float)v.im;
  const __bf16 hr = (__bf16)re, hm = (__bf16)im;
  const __bf16 lr = (__bf16)(float)(v.re - (double)(float)hr);
  const __bf16 lm = (__bf16)(float)(v.im - (double)(float)hm);
  if (hi) {
    const size_t r = ((size_t)(row0 + m) * K + k) * 2;
    hi[r] = hr;
    hi[r + 1] = hm;
    lo[r] = lr;
    lo[r + 1] = lm;
  }
  const size_t t = (size_t)k * 2 * Mt + 2 * (row0 + m);
  thi[t] = hr;
  thi[t + 1] = hm;
  tlo[t] = lr;
  tlo[t + 1] = lm;
}

__device__ __forceinline__ void put_split(__bf16* __restrict__ Cs, size_t plane, size_t i, float re, float im) {
  const __bf16 rh = (__bf16)re, ih = (__bf16)im;
  Cs[2 * i] = rh;
  Cs[2 * i + 1] = ih;
  Cs[plane + 2 * i] = (__bf16)(re - (float)rh);
  Cs[plane + 2 * i + 1] = (__bf16)(im - (float)ih);
}

// Coefficients of (H - eps) p projected, for one expand over the stacked rows
// [KB (Ma rows); Psi (Mb rows)], from the split partials of c_a = <beta_a|p>
// and of <psi_b|q_loc>, q_loc the local part of (H - eps) p:
//   rows a: D c_a;  rows Ma + b: -(<psi_b|q_loc> + sum_a G[a][b] D c_a),
// G[a][b] = <psi_b|beta_a>, so that the Psi rows remove Psi^H of the whole
// (H - eps) p. One workgroup per column n; output as k_sum_split writes it
// for M_pad = Ma + Mb.
__global__ void k_sum_proj(const Z32* __restrict__ cp_a, int ns_a, const Z32* __restrict__ cp_b, int ns_b,
                           int ncols, int Ma, int Mb, float D, const Z32* __restrict__ G, __bf16* __restrict__ Cs,
                           const int* __restrict__ live) {
  extern __shared__ Z32 ca[];
  const int n = blockIdx.x, Mt = Ma + Mb;
  if (live && n >= *live) return;  // whole workgroup, before its barrier
  const size_t plane = (size_t)ncols * Mt * 2, row = (size_t)n * Mt;
  for (int a = threadIdx.x; a < Ma; a += blockDim.x) {
    float re = 0.f, im = 0.f;
    for (int s = 0; s < ns_a; ++s) {
      const Z32 v = cp_a[((size_t)s * ncols + n) * Ma + a];
      re += v.re;
      im += v.im;
    }
    ca[a] = zmk(D * re, D * im);
    put_split(Cs, plane, row + a, D * re, D * im);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < Mb; b += blockDim.x) {
    float re = 0.f, im = 0.f;
    for (int s = 0; s < ns_b; ++s) {
      const Z32 v = cp_b[((size_t)s * ncols + n) * Mb + b];
      re += v.re;
      im += v.im;
    }
    for (int a = 0; a < Ma; ++a) {
      const Z32 g = G[(size_t)a * Mb + b], c = ca[a];
      re += g.re * c.re - g.im * c.im;
      im += g.re * c.im + g.im * c.re;
    }
    put_split(Cs, plane, row + Ma + b, -re, -im);
  }
}

}  // namespace

int choose_nsplit_bf16(int M_pad, int ncols, int K, int target) {
  if (target <= 0) target = kBf16TargetGroups;
  const int base = ((M_pad + kWM - 1) / kWM) * ((ncols + kWN - 1) / kWN);
  int ns = (target + base - 1) / base;
  const int maxs = K / 256 > 0 ? K / 256 : 1;
  if (ns > maxs) ns = maxs;
  if (ns < 1) ns = 1;
  return ns;
}

void launch_split_bf16(const Z64* A, int M, int K, __bf16* hi, __bf16* lo, __bf16* thi, __bf16* tlo, hipStream_t st) {
  launch_split_bf16_rows(A, M, K, 0, M, hi, lo, thi, tlo, st);
}

void launch_split_bf16_rows(const Z64* A, int M, int K, int row0, int Mt, __bf16* hi, __bf16* lo, __bf16* thi,
                            __bf16* tlo, hipStream_t st) {
  const size_t n = (size_t)M * K;
  if (n == 0) return;
  k_split_rows<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(A, M, K, row0, Mt, hi, lo, thi, tlo);
}

void launch_sum_proj32(const Z32* cp_a, int ns_a, const Z32* cp_b, int ns_b, int ncols, int Ma, int Mb, float D,
                       const Z32* G, __bf16* Cs, hipStream_t st, const int* live) {
  if (ncols <= 0) return;
  k_sum_proj<<<ncols, 256, (size_t)Ma * sizeof(Z32), st>>>(cp_a, ns_a, cp_b, ns_b, ncols, Ma, Mb, D, G, Cs, live);
}

void launch_reduce_bf16(const __bf16* Ahi, const __bf16* Alo, int M_pad, const Z32* X, int ldx, const int* xidx,
                        int ncols, int K, Z32* cpart, int nsplit, hipStream_t st, const int* live) {
  if (ncols <= 0) return;
  int kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 31) / 32 * 32;  // whole K steps of 32 complex; K is a multiple of 64
  const int nmb = (M_pad + kWM - 1) / kWM, nnb = (ncols + kWN - 1) / kWN;
  const int groups = (nnb * nsplit + 7) / 8;  // groups of 8 (column block, split) pairs, one per XCD
  k_reduce_bf16w<<<groups * 8 * nmb, kThreads8, 0, st>>>(Ahi, Alo, M_pad, X, ldx, xidx, ncols, K, kchunk, cpart,
                                                          nmb, nnb, nsplit, live);
}

void launch_sum_parts32(const Z32* cpart, int nsplit, int ncols, int M_pad, float scale, __bf16* Cs,
                        hipStream_t st, const int* live) {
  const int total = ncols * M_pad;
  if (total <= 0) return;
  k_sum_split<<<(total + 255) / 256, 256, 0, st>>>(cpart, nsplit, ncols, M_pad, scale, Cs, live);
}

void launch_expand_bf16(const __bf16* ATh, const __bf16* ATl, int M_pad, const __bf16* Cs, Z32* Y, int ldy,
                        const int* yidx, int ncols, int K, int variant, hipStream_t st, Z32* P, const double* beta,
                        const int* live) {
  if (ncols <= 0) return;
  // linear grid: ceil(row blocks / 8) groups x 8 XCD slots x column blocks
  auto grid = [&](int rows, int cols) {
    const int nkb = (K + rows - 1) / rows, nnb = (ncols + cols - 1) / cols;
    return std::make_pair((unsigned)(((nkb + 7) / 8) * 8 * nnb), nnb);
  };
  if (variant == 1) {
    const auto g = grid(128, kEN);
    if (P)
      k_expand_bf16s<2, true, 2><<<g.first, kThreads8, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P, beta,
                                                                g.second, live);
    else
      k_expand_bf16s<2, false, 2><<<g.first, kThreads8, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P,
                                                                 beta, g.second, live);
  } else if (variant == 2) {
    const auto g = grid(kET, 64);
    if (P)
      k_expand_bf16s<4, true, 1><<<g.first, 256, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P, beta,
                                                          g.second, live);
    else
      k_expand_bf16s<4, false, 1><<<g.first, 256, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P, beta,
                                                           g.second, live);
  } else {
    const auto g = grid(kET, kEN);
    if (P)
      k_expand_bf16s<4, true, 2><<<g.first, kThreads8, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P, beta,
                                                                g.second, live);
    else
      k_expand_bf16s<4, false, 2><<<g.first, kThreads8, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P,
                                                                 beta, g.second, live);
  }
}

}  // namespace stern
