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
#include <type_traits>
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

constexpr int kWM = 128;  // reduce: rows of A per workgroup (4 row groups of 32)
constexpr int kWN = 128;  // reduce: columns per workgroup

// C[n][m] partial over this split's K range = sum_k conj(A[m][k]) X[xidx[n]][k].
// 4 WN waves: wave (wm, wn) owns rows [32 wm, 32 wm + 32) and columns
// [CW wn, CW wn + CW), CW = 128 / WN, of the 128 x 128 tile. A K step covers 32
// complex, two MFMA sub-steps of 16. Both operand slices of a step go through
// double-buffered LDS tiles, [sub-step][row or column][4 chunks of 16 bytes]: the
// 128 x 32 slice of X, split into bf16 hi/lo as it is stored, and the 128 x 32
// slice of A (hi, lo). Chunk g of row r sits at g ^ ((r >> 2) & 3), so that the 16
// consecutive rows of one fragment read at one chunk index cover all banks. Each
// step's slices are loaded into registers two steps ahead of their products
// (during the step before) and stored after the current step's products, one
// barrier per step; every load is unconditional (rows and columns out of range
// read valid data whose products are never stored). Re C = A . X and Im C = A' . X
// along the interleaved reduction index, with A' = (-a_im, a_re) formed from A in
// registers.
// Workgroups are numbered so that the row blocks of one (column block, split)
// pair get consecutive slots of one XCD (the hardware hands workgroup L to XCD
// L mod 8): they run together and share that pair's slice of X through the
// XCD's L2 instead of each fetching it from HBM.
template <int WN>
__global__ __launch_bounds__(256 * WN) void k_reduce_bf16w(const __bf16* __restrict__ Ahi,
                                                           const __bf16* __restrict__ Alo, int M_pad,
                                                           const Z32* __restrict__ X, int ldx,
                                                           const int* __restrict__ xidx, int ncols, int K, int kchunk,
                                                           Z32* __restrict__ cpart, int nmb, int nnb, int nsplit,
                                                           const int* __restrict__ ncount) {
  constexpr int NT = 256 * WN, CW = kWN / WN, NBW = CW / 16;
  constexpr int TPC = NT / kWN, CPT = 32 / TPC;  // X staging: threads per column, complex per thread
  constexpr int PA = 2 * kWM * 8 / NT;            // A staging: 16-byte pieces per thread (hi and lo)
  static_assert(CPT % 4 == 0 && PA * NT == 2 * kWM * 8, "whole staging units per thread");
  __shared__ bf16x8 xs[2][2][2][kWN * 4];  // [buffer][hi, lo][sub-step][column * 4 + chunk]
  __shared__ bf16x8 sa[2][2][2][kWM * 4];  // [buffer][hi, lo][sub-step][row * 4 + chunk]
  const int L = blockIdx.x, slot = L >> 3;
  const int mb = slot % nmb, rest = (slot / nmb) * 8 + (L & 7);
  if (rest >= nnb * nsplit) return;  // padding of the last group of XCD slots; no barrier passed yet
  const int nlive = ncount ? min(ncols, *ncount) : ncols;  // ncols stays the stride of the partials
  if ((rest % nnb) * kWN >= nlive) return;  // no live column in this block; no barrier passed yet
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int wm = wave & 3, wn = wave >> 2;
  const int n0 = (rest % nnb) * kWN;
  const int split = rest / nnb;
  const int m0 = mb * kWM + wm * 32;
  const bool live = m0 < M_pad;  // wave-uniform: rows past M_pad (M_pad is a multiple of 64) do no products
  const int kb = split * kchunk;
  const int ke = min(K, kb + kchunk);
  f32x4 cre[2][NBW], cim[2][NBW];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      cre[bi][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      cim[bi][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  if (kb < ke) {  // uniform over the workgroup
    // X staging: thread -> (column tn, CPT complex from index CPT tq of the step)
    const int tn = threadIdx.x / TPC, tq = threadIdx.x % TPC;
    const int xcol = min(n0 + tn, nlive - 1);
    const Z32* xrow = X + (size_t)(xidx ? xidx[xcol] : xcol) * ldx + CPT * tq;
    float4 xv[CPT / 2];
    auto load_x = [&](int kc) {
      const float4* src = reinterpret_cast<const float4*>(xrow + kc);
#pragma unroll
      for (int t = 0; t < CPT / 2; ++t) xv[t] = src[t];
    };
    auto put_x = [&](int buf) {
#pragma unroll
      for (int h = 0; h < CPT / 4; ++h) {
        const int G = (CPT / 4) * tq + h;  // group of 4 complex within the step
        const Z32 v[4] = {zmk(xv[2 * h].x, xv[2 * h].y), zmk(xv[2 * h].z, xv[2 * h].w),
                          zmk(xv[2 * h + 1].x, xv[2 * h + 1].y), zmk(xv[2 * h + 1].z, xv[2 * h + 1].w)};
        bf16x8 hi, lo;
        split_z4(v, hi, lo);
        xs[buf][0][G >> 2][tn * 4 + ((G & 3) ^ ((tn >> 2) & 3))] = hi;
        xs[buf][1][G >> 2][tn * 4 + ((G & 3) ^ ((tn >> 2) & 3))] = lo;
      }
    };
    // A staging: piece p = threadIdx.x + NT j is chunk p & 7 (of 8 per row and step) of row
    // (p >> 3) % 128 of the hi (p < 1024) or lo half; rows past M_pad repeat row M_pad - 1
    bf16x8 av[PA];
    auto load_a = [&](int kc) {
#pragma unroll
      for (int j = 0; j < PA; ++j) {
        const int p = threadIdx.x + NT * j, q = p & 1023;
        const __bf16* src = p < 1024 ? Ahi : Alo;
        av[j] = *reinterpret_cast<const bf16x8*>(src + (size_t)min(mb * kWM + (q >> 3), M_pad - 1) * 2 * K +
                                                 2 * kc + 8 * (q & 7));
      }
    };
    auto put_a = [&](int buf) {
#pragma unroll
      for (int j = 0; j < PA; ++j) {
        const int p = threadIdx.x + NT * j, q = p & 1023, r = q >> 3, c = q & 7;
        sa[buf][p < 1024 ? 0 : 1][c >> 2][r * 4 + ((c & 3) ^ ((r >> 2) & 3))] = av[j];
      }
    };
    const int sw = (l16 >> 2) & 3;  // swizzle of the fragment rows and columns this lane reads
    load_x(kb);
    load_a(kb);
    put_x(0);
    put_a(0);
    load_x(min(kb + 32, ke - 32));
    load_a(min(kb + 32, ke - 32));
    __syncthreads();
    // The K loop is instantiated with and without the products, so that the
    // accumulators are updated in place on every path.
    auto steps = [&](auto with_products) {
      int buf = 0;
      for (int kc = kb; kc < ke; kc += 32) {
        if constexpr (decltype(with_products)::value) {
#pragma unroll
          for (int kk = 0; kk < 2; ++kk) {
            bf16x8 a_hi[2], a_lo[2], b_hi[2], b_lo[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) {
              const int r = wm * 32 + bi * 16 + l16;
              a_hi[bi] = sa[buf][0][kk][r * 4 + (g ^ sw)];
              a_lo[bi] = sa[buf][1][kk][r * 4 + (g ^ sw)];
              b_hi[bi] = rot_neg(a_hi[bi]);
              b_lo[bi] = rot_neg(a_lo[bi]);
            }
#pragma unroll
            for (int nb = 0; nb < NBW; ++nb) {
              const int col = wn * CW + nb * 16 + l16;
              const bf16x8 x_hi = xs[buf][0][kk][col * 4 + (g ^ sw)];
              const bf16x8 x_lo = xs[buf][1][kk][col * 4 + (g ^ sw)];
#pragma unroll
              for (int bi = 0; bi < 2; ++bi) {
                cre[bi][nb] = mfma(a_hi[bi], x_hi, cre[bi][nb]);
                cre[bi][nb] = mfma(a_hi[bi], x_lo, cre[bi][nb]);
                cre[bi][nb] = mfma(a_lo[bi], x_hi, cre[bi][nb]);
                cim[bi][nb] = mfma(b_hi[bi], x_hi, cim[bi][nb]);
                cim[bi][nb] = mfma(b_hi[bi], x_lo, cim[bi][nb]);
                cim[bi][nb] = mfma(b_lo[bi], x_hi, cim[bi][nb]);
              }
            }
          }
        }
        // keeps the split of the next step's X below the products: hoisted among them, it would
        // wait on loads issued just before
        __builtin_amdgcn_sched_barrier(0);
        put_x(buf ^ 1);  // the next step's slices (the last step stores a copy of itself, unused)
        put_a(buf ^ 1);
        __syncthreads();
        load_x(min(kc + 64, ke - 32));
        load_a(min(kc + 64, ke - 32));
        buf ^= 1;
      }
    };
    if (!live) {  // loads and barriers only
      steps(std::false_type{});
      return;
    }
    steps(std::true_type{});
  }
  if (!live) return;
  // D[i][j]: column j = lane % 16 (vector), row i = 4 (lane / 16) + r
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    const int n = n0 + wn * CW + nb * 16 + l16;
    if (n >= nlive) continue;
    Z32* dst = cpart + ((size_t)split * ncols + n) * M_pad;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[m0 + 16 * bi + 4 * g + r] = zmk(cre[bi][nb][r], cim[bi][nb][r]);
  }
}

// Blocked layout of the expand's operands: element (m, row) of an M x nrows
// complex matrix (M a multiple of 16) at [m / 16][row][m % 16], interleaved re, im.
// A^T (rows k) and the coefficients C (rows n) are kept this way, so that the 16 m
// of one expand step for one row are 64 contiguous bytes, and the step's rows of a
// tile one contiguous stretch.
__host__ __device__ __forceinline__ size_t blk_index(int m, int row, int nrows) {
  return ((size_t)(m >> 4) * nrows + row) * 32 + 2 * (m & 15);
}

// C = scale * sum of the split partials, as bf16 hi and lo of (c_re, c_im):
// Cs[0], Cs[1], each M_pad x ncols in the blocked layout.
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
  const size_t plane = (size_t)total * 2, o = blk_index(i % M_pad, i / M_pad, ncols);
  const __bf16 rh = (__bf16)re, ih = (__bf16)im;
  Cs[o] = rh;
  Cs[o + 1] = ih;
  Cs[plane + o] = (__bf16)(re - (float)rh);
  Cs[plane + o + 1] = (__bf16)(im - (float)ih);
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

// Y[yidx[n]][k] += sum_m A[m][k] C[n][m], with A^T and C in the blocked layouts
// (blk_index) and split hi/lo. PUPD: Y is left as it is and the sum goes into the
// search direction instead, P[s] = (Y[s] + A C) + beta[s] P[s] (s = yidx[n]), the CG
// direction update from the projected z.
// Tile: RK = 64 KB rows k x RN = 16 NB WC columns, 4 WC waves; wave (wk, wc) owns
// rows [16 KB wk, 16 KB (wk + 1)) and columns [16 NB wc, 16 NB (wc + 1)). One step
// covers 16 complex m: the step's A^T rows and C columns are contiguous stretches
// of the blocked layouts, loaded coalesced into registers one step ahead, stored
// to a double-buffered LDS tile (one barrier per step) and read as MFMA fragments
// from there. Rows of the LDS tile are 64 bytes (4 chunks of 16); chunk c of row r
// sits at chunk c ^ ((r >> 2) & 3), so the 16 lanes that read one fragment column
// cover all LDS banks once. Every global load is unconditional (rows past K and
// columns past the live count read valid data that is never stored), so the next
// step's loads stay in flight across this step's products.
// Re(a c) = a . (c_re, -c_im), Im(a c) = a . (c_im, c_re).
// Workgroups are numbered so that the column blocks of one row block k get
// consecutive slots of one XCD (workgroup L runs on XCD L mod 8) and share
// that block's rows of A through the XCD's L2.
__device__ __forceinline__ int swz(int r, int c) { return r * 4 + (c ^ ((r >> 2) & 3)); }

template <int KB, int NB, int WC, bool PUPD>
__global__ __launch_bounds__(256 * WC) void k_expand_bf16s(const __bf16* __restrict__ ATh,
                                                           const __bf16* __restrict__ ATl, int M_pad, int K,
                                                           const __bf16* __restrict__ Cs, Z32* __restrict__ Y,
                                                           int ldy, const int* __restrict__ yidx, int ncols,
                                                           Z32* __restrict__ P, const double* __restrict__ beta,
                                                           int nnb, const int* __restrict__ live) {
  constexpr int RK = 64 * KB, RN = 16 * NB * WC, NT = 256 * WC;
  constexpr int PA = 8 * RK / NT, PC = 8 * RN / NT;  // 16-byte pieces (hi and lo) per thread and step
  static_assert(PA >= 1 && PC >= 1 && PA * NT == 8 * RK && PC * NT == 8 * RN, "whole pieces per thread");
  __shared__ bf16x8 as[2][2 * RK * 4];  // [buffer][hi, lo][row k * 4 + chunk]
  __shared__ bf16x8 cs[2][2 * RN * 4];  // [buffer][hi, lo][column n * 4 + chunk]
  const int nlive = live ? min(ncols, *live) : ncols;  // ncols stays the stride of C
  const int L = blockIdx.x, slot = L >> 3;
  const int nbk = slot % nnb, kblk = (slot / nnb) * 8 + (L & 7);
  const int kt0 = kblk * RK, nt0 = nbk * RN;
  if (kt0 >= K || nt0 >= nlive) return;  // whole workgroup, before any barrier
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int l16 = lane & 15, g = lane >> 4;
  const int wk = wave & 3, wc = wave >> 2;
  const bool wlive = nt0 + 16 * NB * wc < nlive;  // wave-uniform: a wave with no live column does no products
  // staging: piece p = threadIdx.x + NT j of the step's A^T tile is chunk p & 3 of row (p >> 2) % RK of
  // the hi (p < 4 RK) or lo half (rows past K repeat row K - 1), and likewise for the C tile (columns
  // past the live count repeat the last live one). Offsets are formed where used, to save registers.
  const size_t cplane = (size_t)ncols * M_pad * 2;
  const size_t astep = (size_t)K * 32, cstep = (size_t)ncols * 32;
  bf16x8 ra[PA], rc[PC];
  auto gload = [&](int st) {
#pragma unroll
    for (int j = 0; j < PA; ++j) {
      const int p = threadIdx.x + NT * j, q = p % (4 * RK);
      const __bf16* src = p < 4 * RK ? ATh : ATl;
      ra[j] = *reinterpret_cast<const bf16x8*>(src + st * astep + (size_t)min(kt0 + (q >> 2), K - 1) * 32 +
                                               8 * (q & 3));
    }
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      const int p = threadIdx.x + NT * j, q = p % (4 * RN);
      rc[j] = *reinterpret_cast<const bf16x8*>(Cs + (p < 4 * RN ? 0 : cplane) + st * cstep +
                                               (size_t)min(nt0 + (q >> 2), nlive - 1) * 32 + 8 * (q & 3));
    }
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int j = 0; j < PA; ++j) {
      const int p = threadIdx.x + NT * j, q = p % (4 * RK);
      as[b][(p < 4 * RK ? 0 : 4 * RK) + swz(q >> 2, q & 3)] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < PC; ++j) {
      const int p = threadIdx.x + NT * j, q = p % (4 * RN);
      cs[b][(p < 4 * RN ? 0 : 4 * RN) + swz(q >> 2, q & 3)] = rc[j];
    }
  };
  f32x4 dre[KB][NB], dim_[KB][NB];
#pragma unroll
  for (int bi = 0; bi < KB; ++bi)
#pragma unroll
    for (int bj = 0; bj < NB; ++bj) {
      dre[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
      dim_[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  const int nsteps = M_pad >> 4;
  gload(0);
  lstore(0);
  __syncthreads();
  gload(min(1, nsteps - 1));
  const int sw = (l16 >> 2) & 3;  // swizzle of the fragment rows this lane reads (rows 16 q + l16)
  // The step loop is instantiated twice, with and without the products, so that the
  // accumulators are updated in place on every path (a branch around the products
  // inside the loop makes the compiler copy them each step).
  auto steps = [&](auto with_products) {
    for (int st = 0; st < nsteps; ++st) {
      const int b = st & 1;
      if constexpr (decltype(with_products)::value) {
        bf16x8 a_hi[KB], a_lo[KB];
#pragma unroll
        for (int bi = 0; bi < KB; ++bi) {
          const int r = 16 * (KB * wk + bi) + l16;
          a_hi[bi] = as[b][r * 4 + (g ^ sw)];
          a_lo[bi] = as[b][4 * RK + r * 4 + (g ^ sw)];
        }
#pragma unroll
        for (int bj = 0; bj < NB; ++bj) {
          const int r = 16 * (NB * wc + bj) + l16;
          const bf16x8 ch = cs[b][r * 4 + (g ^ sw)], cl = cs[b][4 * RN + r * 4 + (g ^ sw)];
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
          if constexpr (NB > 4) __builtin_amdgcn_sched_barrier(0);  // one column group's fragments at a time
        }
      }
      lstore(b ^ 1);  // the next step's tile (the last step stores a copy of itself, unused)
      __syncthreads();
      gload(min(st + 2, nsteps - 1));
    }
  };
  if (!wlive) {  // loads and barriers only
    steps(std::false_type{});
    return;
  }
  steps(std::true_type{});
  // D[i][j]: column j = lane % 16 (vector), rows i = 4 (lane / 16) + r: 4 consecutive k per lane
#pragma unroll
  for (int bj = 0; bj < NB; ++bj) {
    const int n = nt0 + 16 * (NB * wc + bj) + l16;
    if (n >= nlive) continue;
    const size_t row = (size_t)(yidx ? yidx[n] : n);
    Z32* y = Y + row * ldy;
    float bt = 0.f;
    if constexpr (PUPD) bt = (float)beta[row];
#pragma unroll
    for (int bi = 0; bi < KB; ++bi) {
      const int k = kt0 + 16 * (KB * wk + bi) + 4 * g;
      if (k >= K) continue;  // K is a multiple of 64: a group of 16 rows is wholly in or out
      float4* p = reinterpret_cast<float4*>(y + k);
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
        float4* d = reinterpret_cast<float4*>(P + row * ldy + k);
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
// matrix of Mt rows, in row layout [Mt][2K] (skipped when hi is null, interleaved
// re, im) and transposed in the blocked layout of the expand (blk_index(m, k, K))
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
  const size_t t = blk_index(row0 + m, k, K);
  thi[t] = hr;
  thi[t + 1] = hm;
  tlo[t] = lr;
  tlo[t + 1] = lm;
}

// hi and lo of (re, im) at element offset o of the two planes of Cs
__device__ __forceinline__ void put_split(__bf16* __restrict__ Cs, size_t plane, size_t o, float re, float im) {
  const __bf16 rh = (__bf16)re, ih = (__bf16)im;
  Cs[o] = rh;
  Cs[o + 1] = ih;
  Cs[plane + o] = (__bf16)(re - (float)rh);
  Cs[plane + o + 1] = (__bf16)(im - (float)ih);
}

// Coefficients of the projected (H - eps) p over the stacked rows [P_c KB (Ma); Psi (Mb)] from
// the split partials of <beta_a|p> and of <psi_b|q_loc>, q_loc the local part of (H - eps) p:
// rows a: D <beta_a|p>; rows Ma + b: -<psi_b|q_loc>. With P_c beta_a in the stacked matrix the
// Psi rows need not remove Psi^H of the KB term. Output as k_sum_split writes it for M_pad = Ma + Mb.
__global__ void k_sum_proj(const Z32* __restrict__ cp_a, int ns_a, const Z32* __restrict__ cp_b, int ns_b,
                           int ncols, int Ma, int Mb, float D, __bf16* __restrict__ Cs,
                           const int* __restrict__ live) {
  const int Mt = Ma + Mb;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncols * Mt) return;
  const int n = i / Mt, r = i - n * Mt;
  if (live && n >= *live) return;
  const bool kb = r < Ma;
  const Z32* src = kb ? cp_a + (size_t)n * Ma + r : cp_b + (size_t)n * Mb + (r - Ma);
  const size_t stride = (size_t)ncols * (kb ? Ma : Mb);
  const int ns = kb ? ns_a : ns_b;
  float re = 0.f, im = 0.f;
  for (int s = 0; s < ns; ++s) {
    const Z32 v = src[s * stride];
    re += v.re;
    im += v.im;
  }
  const float f = kb ? D : -1.f;
  put_split(Cs, (size_t)ncols * Mt * 2, blk_index(r, n, ncols), f * re, f * im);
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
                       __bf16* Cs, hipStream_t st, const int* live) {
  const int total = ncols * (Ma + Mb);
  if (total <= 0) return;
  k_sum_proj<<<(total + 255) / 256, 256, 0, st>>>(cp_a, ns_a, cp_b, ns_b, ncols, Ma, Mb, D, Cs, live);
}

void launch_reduce_bf16(const __bf16* Ahi, const __bf16* Alo, int M_pad, const Z32* X, int ldx, const int* xidx,
                        int ncols, int K, Z32* cpart, int nsplit, hipStream_t st, const int* live) {
  if (ncols <= 0) return;
  int kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + 31) / 32 * 32;  // whole K steps of 32 complex; K is a multiple of 64
  const int nmb = (M_pad + kWM - 1) / kWM, nnb = (ncols + kWN - 1) / kWN;
  const int groups = (nnb * nsplit + 7) / 8;  // groups of 8 (column block, split) pairs, one per XCD
  // 16 waves of 32 x 32 (as fast as 8 waves of 32 x 64 at these shapes, and 40% fewer registers)
  k_reduce_bf16w<4><<<groups * 8 * nmb, 1024, 0, st>>>(Ahi, Alo, M_pad, X, ldx, xidx, ncols, K, kchunk, cpart, nmb,
                                                       nnb, nsplit, live);
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
  auto go = [&](auto kern, int rows, int cols, int threads) {
    const int nkb = (K + rows - 1) / rows, nnb = (ncols + cols - 1) / cols;
    kern<<<(unsigned)(((nkb + 7) / 8) * 8 * nnb), threads, 0, st>>>(ATh, ATl, M_pad, K, Cs, Y, ldy, yidx, ncols, P,
                                                                   beta, nnb, live);
  };
  if (variant == 1) {  // 128 x 128 tile, 16 waves of 32 x 32
    if (P) go(k_expand_bf16s<2, 2, 4, true>, 128, 128, 1024);
    else go(k_expand_bf16s<2, 2, 4, false>, 128, 128, 1024);
  } else if (variant == 2) {  // 128 x 128 tile, 8 waves of 32 x 64
    if (P) go(k_expand_bf16s<2, 4, 2, true>, 128, 128, 512);
    else go(k_expand_bf16s<2, 4, 2, false>, 128, 128, 512);
  } else {  // 256 x 128 tile, 8 waves of 64 x 64
    if (P) go(k_expand_bf16s<4, 4, 2, true>, 256, 128, 512);
    else go(k_expand_bf16s<4, 4, 2, false>, 256, 128, 512);
  }
}

}  // namespace stern
