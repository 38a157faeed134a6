// Pruned 3-D FFT kernels of the H apply, the right-hand side and the density
// response. A vector on the plane-wave sphere goes through
//   x pass:  per x-pencil column (n_y, n_z) of the sphere, a length-N DFT along x
//   yz pass: per plane ix, a 2-D DFT over the columns' (iy, iz) positions
// so HBM only ever holds the sphere and its columns, never the N^3 box.
//
// Every length-N transform is two Stockham stages N = R1 * R2 done in
// registers with one LDS exchange between them. The first stage of a pass
// gathers straight from global memory and the last scatters straight to it.
// In the yz pass of the H apply the inverse transform along z ends with the
// radix-R2 stage over the elements {j + r R1}; the forward transform is run
// with the reversed plan (R2 first), whose first stage consumes exactly those
// elements, so inverse stage 2, the V_loc multiply and forward stage 1 happen
// in registers without an LDS round trip.
#include <algorithm>
#include <mutex>

#include "fft_dev.hpp"
#include "kernels.hpp"

namespace stern {

namespace {

// threads of a yz-plane workgroup: enough for one item per thread in the row
// stages, capped so that the FP64 kernels keep 2 waves per SIMD (256 VGPRs)
template <int N, class T = double>
constexpr int plane_nt() {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  constexpr int m = N * (R1 > R2 ? R1 : R2);
  constexpr int r = (m + 63) / 64 * 64;
  constexpr int cap = sizeof(T) == 8 ? 512 : 768;
  return r < 256 ? 256 : (r > cap ? cap : r);
}
constexpr int kXThreads = 256;

template <class T>
__device__ __forceinline__ const Z<T>* twtab(const FftGeom& g);
template <>
__device__ __forceinline__ const Z64* twtab<double>(const FftGeom& g) { return g.tw64; }
template <>
__device__ __forceinline__ const Z32* twtab<float>(const FftGeom& g) { return g.tw32; }

// One radix-R Stockham stage of length-N transforms over F lines. Item (f, j)
// with j < N/R loads v[r] = ld(f, j, r), applies exp(DIR 2 pi i r j / N) when
// TWID, transforms and stores st(f, j, r, v[r]). LINE_FAST orders items with
// the line index fastest. SYNC puts a barrier between all loads and all
// stores (for stages that read and write different LDS positions).
template <int N, int R, int DIR, bool TWID, bool SYNC, bool LINE_FAST, int NT, int MAXF, class T, class Ld,
          class St>
__device__ __forceinline__ void stage(int F, Ld ld, St st, const Z<T>* __restrict__ tw) {
  constexpr int J = N / R;
  const int tid = threadIdx.x;
  // item -> (line f, index j)
  auto line_of = [F](int it) { return LINE_FAST ? it % F : it / J; };
  auto idx_of = [F](int it) { return LINE_FAST ? it / F : it % J; };
  if constexpr (SYNC) {
    constexpr int MAXIT = (MAXF * J + NT - 1) / NT;
    Z<T> v[MAXIT][R];
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int it = tid + k * NT;
      if (it < F * J) {
        const int f = line_of(it), j = idx_of(it);
#pragma unroll
        for (int r = 0; r < R; ++r) v[k][r] = ld(f, j, r);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int it = tid + k * NT;
      if (it < F * J) {
        const int f = line_of(it), j = idx_of(it);
        if constexpr (TWID) {
#pragma unroll
          for (int r = 1; r < R; ++r) v[k][r] = v[k][r] * twid<DIR>(tw, r * j);
        }
        dft<R, DIR>(v[k]);
#pragma unroll
        for (int r = 0; r < R; ++r) st(f, j, r, v[k][r]);
      }
    }
  } else {
    for (int it = tid; it < F * J; it += NT) {
      const int f = line_of(it), j = idx_of(it);
      Z<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = ld(f, j, r);
      if constexpr (TWID) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = v[r] * twid<DIR>(tw, r * j);
      }
      dft<R, DIR>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) st(f, j, r, v[r]);
    }
  }
}

// ---------------------------------------------------------------- x pass ----
// A workgroup takes CB consecutive x-pencil columns. Their sphere coefficients are one
// contiguous range of the vector (column order), so the sphere side of both passes is
// a single coalesced sweep of that range through LDS: each coefficient finds its
// column by a binary search over the block's column starts (kept in LDS; padding
// columns hold INT_MAX) and its x from the column's smallest n_x.
template <int N, class T>
struct XBlock {
  static constexpr int CB = col_block<T>(), LDX = N + 1;
  int s0, s1;  // sphere range of the block
  __device__ __forceinline__ void load(const FftGeom& g, int c0, int* bs, int* bx) {
    const int tid = threadIdx.x;
    if (tid < CB) {
      const int c = c0 + tid, len = g.col_len[c];
      bs[tid] = len > 0 ? g.col_start[c] : 0x7fffffff;
      bx[tid] = g.col_xmin[c];
    }
  }
  // after a barrier that follows load(): the block's range. Columns are padded to whole
  // blocks of the widest block size, so a narrower block may hold padding only: its range
  // is empty (starting it at the padding marker would overflow the sphere index).
  __device__ __forceinline__ void range(const FftGeom& g, int c0, const int* bs) {
    if (bs[0] == 0x7fffffff) {
      s0 = s1 = 0;
      return;
    }
    s0 = bs[0];
    s1 = s0;
#pragma unroll
    for (int cc = 0; cc < CB; ++cc)
      if (bs[cc] != 0x7fffffff) s1 = g.col_start[c0 + cc] + g.col_len[c0 + cc];
  }
  // LDS slot (column cc, x) of sphere index gi in [s0, s1)
  __device__ __forceinline__ int slot(int gi, const int* bs, const int* bx) const {
    int cc = 0;
#pragma unroll
    for (int step = CB / 2; step > 0; step >>= 1)
      if (bs[cc + step] <= gi) cc += step;
    const int nx = bx[cc] + (gi - bs[cc]);
    return cc * LDX + (nx < 0 ? nx + N : nx);
  }
};

// inverse: sphere coefficients -> pencils [vec][ix][ncol_pad]
template <int N, class T>
__global__ __launch_bounds__(kXThreads) void k_xinv(const Z<T>* __restrict__ sph, const int* __restrict__ vidx,
                                                    Z<T>* __restrict__ pen, FftGeom g) {
  using B = XBlock<N, T>;
  constexpr int CB = B::CB, LDX = B::LDX;
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  __shared__ Z<T> P[CB * LDX];
  __shared__ int bs[CB], bx[CB];
  if (g.live && (int)blockIdx.y >= *g.live) return;  // vector not live (whole workgroup, before any barrier)
  const Z<T>* tw = twtab<T>(g);
  const int c0 = blockIdx.x * CB;
  const int vec = vidx ? vidx[blockIdx.y] : blockIdx.y;
  const Z<T>* src = sph + (size_t)vec * g.npw_pad;
  B blk;
  blk.load(g, c0, bs, bx);
  for (int i = threadIdx.x; i < CB * LDX; i += kXThreads) P[i] = zmk(T(0), T(0));
  __syncthreads();
  blk.range(g, c0, bs);
  for (int gi = blk.s0 + (int)threadIdx.x; gi < blk.s1; gi += kXThreads) P[blk.slot(gi, bs, bx)] = src[gi];
  __syncthreads();
  // stage 1 in place (all loads before the barrier inside, then the stores)
  stage<N, R1, +1, false, true, true, kXThreads, CB>(
      CB, [&](int cc, int j, int r) { return P[cc * LDX + j + r * R2]; },
      [&](int cc, int j, int r, Z<T> v) { P[cc * LDX + j * R1 + r] = v; }, tw);
  __syncthreads();
  Z<T>* dst = pen + (size_t)vec * N * g.ncol_pad + c0;
  const int ld = g.ncol_pad;
  stage<N, R2, +1, true, false, true, kXThreads, CB>(
      CB, [&](int cc, int j, int r) { return P[cc * LDX + j + r * R1]; },
      [&](int cc, int j, int r, Z<T> v) { dst[(size_t)(j + r * R1) * ld + cc] = v; }, tw);
}

// forward: pencils -> sphere; MODE 0 plain, 1 adds (|G|^2/2 - eps) pin, 2 scales
template <int N, class T, int MODE>
__global__ __launch_bounds__(kXThreads) void k_xfwd(const Z<T>* __restrict__ pen, const int* __restrict__ vidx,
                                                    Z<T>* __restrict__ out, const Z<T>* __restrict__ pin,
                                                    const double* __restrict__ eps, double scale, FftGeom g) {
  using B = XBlock<N, T>;
  constexpr int CB = B::CB, LDX = B::LDX;
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  __shared__ Z<T> P[CB * LDX];
  __shared__ int bs[CB], bx[CB];
  if (g.live && (int)blockIdx.y >= *g.live) return;  // vector not live (whole workgroup, before any barrier)
  const Z<T>* tw = twtab<T>(g);
  const int c0 = blockIdx.x * CB;
  const int vec = vidx ? vidx[blockIdx.y] : blockIdx.y;
  const Z<T>* src = pen + (size_t)vec * N * g.ncol_pad + c0;
  const int ld = g.ncol_pad;
  B blk;
  blk.load(g, c0, bs, bx);
  stage<N, R1, -1, false, false, true, kXThreads, CB>(
      CB, [&](int cc, int j, int r) { return src[(size_t)(j + r * R2) * ld + cc]; },
      [&](int cc, int j, int r, Z<T> v) { P[cc * LDX + j * R1 + r] = v; }, tw);
  __syncthreads();
  // stage 2 in place: each item reads and writes the same slots x = j + R1 r
  stage<N, R2, -1, true, false, true, kXThreads, CB>(
      CB, [&](int cc, int j, int r) { return P[cc * LDX + j + r * R1]; },
      [&](int cc, int j, int r, Z<T> v) { P[cc * LDX + j + r * R1] = v; }, tw);
  __syncthreads();
  blk.range(g, c0, bs);
  Z<T>* dst = out + (size_t)vec * g.npw_pad;
  const Z<T>* pv = (MODE == 1) ? pin + (size_t)vec * g.npw_pad : nullptr;
  const T e = (MODE == 1) ? T(eps[vec]) : T(0);
  const T sc = T(scale);
  const double* __restrict__ g2h = g.g2h;
  for (int gi = blk.s0 + (int)threadIdx.x; gi < blk.s1; gi += kXThreads) {
    Z<T> v = P[blk.slot(gi, bs, bx)];
    if (MODE == 1) {
      const T d = T(g2h[gi]) - e;
      const Z<T> pp = pv[gi];
      v = zmk(v.re + d * pp.re, v.im + d * pp.im);
    } else if (MODE == 2) {
      v = zscale(v, sc);
    }
    dst[gi] = v;
  }
  // the row padding [npw, npw_pad) is kept at zero: the GEMMs reduce over it
  if (blockIdx.x == 0)
    for (int k = g.npw + threadIdx.x; k < g.npw_pad; k += kXThreads) dst[k] = zmk(T(0), T(0));
}

// --------------------------------------------------------------- yz pass ----
// Shared pieces. The plane is P[iy * LD + iz]; the active z lines are the
// grid columns iz holding sphere data (iz <= zlo or iz >= zhi); yc[iy * nza + f]
// is the pencil column of (iy, zl[f]) or -1 outside the sphere's disk, laid out
// [iy][f] so that lanes walking the lines read consecutive entries.
template <int N, class T>
struct PlaneCtx {
  static constexpr int LD = N + 1;
  static constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  static constexpr int NT = plane_nt<N, T>();
  Z<T>* P;
  const int* __restrict__ zl;
  const int* __restrict__ yc;
  int nza, zlo, zhi;
  const Z<T>* tw;
  __device__ bool zact(int z) const { return z <= zlo || z >= zhi; }
};

// The twiddle table is copied behind the plane in LDS (N entries); the copy is
// ordered before its first use by the barrier that follows the first stage.
template <int N, class T>
__device__ __forceinline__ const Z<T>* plane_twiddles(unsigned char* smem, const FftGeom& g) {
  Z<T>* t = reinterpret_cast<Z<T>*>(smem) + N * PlaneCtx<N, T>::LD;
  const Z<T>* src = twtab<T>(g);
  for (int i = threadIdx.x; i < N; i += blockDim.x) t[i] = src[i];
  return t;
}

// pencils of one plane -> inverse DFT along y on the active z lines (in LDS)
template <int N, class T>
__device__ __forceinline__ void y_inverse_from_pencils(const PlaneCtx<N, T>& c, const Z<T>* __restrict__ tp) {
  constexpr int LD = PlaneCtx<N, T>::LD, R1 = PlaneCtx<N, T>::R1, R2 = PlaneCtx<N, T>::R2, NT = PlaneCtx<N, T>::NT;
  Z<T>* P = c.P;
  const int* zl = c.zl;
  const int* yc = c.yc;
  const Z<T> zero = zmk(T(0), T(0));
  stage<N, R1, +1, false, false, true, NT, N / 2 + 1>(
      c.nza,
      [&](int f, int j, int r) {
        const int col = yc[(j + r * R2) * c.nza + f];
        Z<T> v = zero;
        if (col >= 0) v = tp[col];
        return v;
      },
      [&](int f, int j, int r, Z<T> v) { P[(j * R1 + r) * LD + zl[f]] = v; }, c.tw);
  __syncthreads();
  stage<N, R2, +1, true, false, true, NT, N / 2 + 1>(
      c.nza, [&](int f, int j, int r) { return P[(j + r * R1) * LD + zl[f]]; },
      [&](int f, int j, int r, Z<T> v) { P[(j + r * R1) * LD + zl[f]] = v; }, c.tw);
  __syncthreads();
}

// forward DFT along y on the active z lines (in LDS) -> pencils of one plane
template <int N, class T>
__device__ __forceinline__ void y_forward_to_pencils(const PlaneCtx<N, T>& c, Z<T>* __restrict__ tp) {
  constexpr int LD = PlaneCtx<N, T>::LD, R1 = PlaneCtx<N, T>::R1, R2 = PlaneCtx<N, T>::R2, NT = PlaneCtx<N, T>::NT;
  Z<T>* P = c.P;
  const int* zl = c.zl;
  const int* yc = c.yc;
  stage<N, R1, -1, false, true, true, NT, N / 2 + 1>(
      c.nza, [&](int f, int j, int r) { return P[(j + r * R2) * LD + zl[f]]; },
      [&](int f, int j, int r, Z<T> v) { P[(j * R1 + r) * LD + zl[f]] = v; }, c.tw);
  __syncthreads();
  stage<N, R2, -1, true, false, true, NT, N / 2 + 1>(
      c.nza, [&](int f, int j, int r) { return P[(j + r * R1) * LD + zl[f]]; },
      [&](int f, int j, int r, Z<T> v) {
        const int col = yc[(j + r * R1) * c.nza + f];
        if (col >= 0) tp[col] = v;
      },
      c.tw);
}

// inverse stage 1 along z on every row (inputs outside the active lines are zero)
template <int N, class T>
__device__ __forceinline__ void z_inverse_stage1(const PlaneCtx<N, T>& c) {
  constexpr int LD = PlaneCtx<N, T>::LD, R1 = PlaneCtx<N, T>::R1, R2 = PlaneCtx<N, T>::R2, NT = PlaneCtx<N, T>::NT;
  Z<T>* P = c.P;
  const Z<T> zero = zmk(T(0), T(0));
  stage<N, R1, +1, false, true, false, NT, N>(
      N,
      [&](int y, int j, int r) {
        const int z = j + r * R2;
        return c.zact(z) ? P[y * LD + z] : zero;
      },
      [&](int y, int j, int r, Z<T> v) { P[y * LD + j * R1 + r] = v; }, c.tw);
  __syncthreads();
}

// LDS of the H-apply plane kernel: the plane, the twiddles and (when it fits
// in 160 KiB) the V_loc plane.
template <int N, class T>
constexpr size_t vloc_lds_bytes(bool with_v) {
  return ((size_t)N * (N + 1) + N) * sizeof(Z<T>) + (with_v ? (size_t)N * (N + 1) * sizeof(T) : 0);
}
template <int N, class T>
constexpr bool vloc_v_in_lds() {
  return vloc_lds_bytes<N, T>(true) <= 160 * 1024;
}

// H apply, in place on the pencils of vectors vidx[b] (b < nvec): for each
// plane, inverse y, inverse z, x V_loc, forward z, forward y.
//
// Persistent and software-pipelined: workgroup w walks the (plane, vector)
// pairs q = w, w + gridDim.x, ... in plane-major order and, while the row
// stages of pair q run, already has the pencil loads of pair q + gridDim.x in
// flight in registers; V_loc(ix, :, :) is re-staged in LDS only when the plane
// changes. Row stages take the row index as the fast lane index, so LDS
// accesses stride by N + 1 elements and avoid bank conflicts.
template <int N, class T>
__global__ __launch_bounds__((plane_nt<N, T>())) void k_plane_vloc(Z<T>* __restrict__ pen, const int* __restrict__ vidx,
                                                             int nvec, const T* __restrict__ v_r, FftGeom g) {
  using C = PlaneCtx<N, T>;
  constexpr int LD = C::LD, R1 = C::R1, R2 = C::R2, NT = C::NT;
  constexpr bool VL = vloc_v_in_lds<N, T>();
  constexpr int MAXA = ((N / 2 + 1) * R2 + NT - 1) / NT;  // first-stage items per thread (nza <= N/2 + 1)
  extern __shared__ unsigned char smem_raw[];
  C c{reinterpret_cast<Z<T>*>(smem_raw), g.zl, g.ycol, g.nza, g.zact_lo, g.zact_hi, plane_twiddles<N, T>(smem_raw, g)};
  Z<T>* P = c.P;
  T* VS = reinterpret_cast<T*>(smem_raw + ((size_t)N * LD + N) * sizeof(Z<T>));
  const int tid = threadIdx.x;
  const int nza = c.nza;
  if (g.live) nvec = min(nvec, *g.live);  // pairs (plane, vector) of the live vectors only
  const long total = (long)N * nvec;
  const Z<T> zero = zmk(T(0), T(0));
  Z<T> pre[MAXA][R1];
  auto prefetch = [&](long q) {
    const int ix = (int)(q / nvec), b = (int)(q - (long)ix * nvec);
    const int vec = vidx ? vidx[b] : b;
    const Z<T>* tp = pen + ((size_t)vec * N + ix) * g.ncol_pad;
#pragma unroll
    for (int k = 0; k < MAXA; ++k) {
      const int it = tid + k * NT;
      const int f = it % nza, j = it / nza;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int cl = (it < nza * R2) ? c.yc[(j + r * R2) * nza + f] : -1;
        Z<T> v = zero;
        if (cl >= 0) v = tp[cl];
        pre[k][r] = v;
      }
    }
  };
  long q = blockIdx.x;
  if (q < total) prefetch(q);
  int cur_ix = -1;
  for (; q < total; q += gridDim.x) {
    const int ix = (int)(q / nvec), b = (int)(q - (long)ix * nvec);
    const int vec = vidx ? vidx[b] : b;
    Z<T>* tp = pen + ((size_t)vec * N + ix) * g.ncol_pad;
    const T* __restrict__ vg = v_r + (size_t)ix * N * N;
    if (VL && ix != cur_ix) {
      for (int i = tid; i < N * N; i += NT) VS[(i / N) * LD + i % N] = vg[i];
    }
    cur_ix = ix;
    // y inverse, stage 1 from the prefetched pencils
#pragma unroll
    for (int k = 0; k < MAXA; ++k) {
      const int it = tid + k * NT;
      if (it < nza * R2) {
        const int f = it % nza, j = it / nza;
        dft<R1, +1>(pre[k]);
#pragma unroll
        for (int r = 0; r < R1; ++r) P[(j * R1 + r) * LD + c.zl[f]] = pre[k][r];
      }
    }
    __syncthreads();
    stage<N, R2, +1, true, false, true, NT, N / 2 + 1>(
        nza, [&](int f, int j, int r) { return P[(j + r * R1) * LD + c.zl[f]]; },
        [&](int f, int j, int r, Z<T> v) { P[(j + r * R1) * LD + c.zl[f]] = v; }, c.tw);
    __syncthreads();
    if (q + gridDim.x < total) prefetch(q + gridDim.x);  // in flight during the row stages
    // z inverse stage 1 (inputs off the active lines are zero)
    stage<N, R1, +1, false, true, true, NT, N>(
        N,
        [&](int y, int j, int r) {
          const int z = j + r * R2;
          Z<T> v = zero;
          if (c.zact(z)) v = P[y * LD + z];
          return v;
        },
        [&](int y, int j, int r, Z<T> v) { P[y * LD + j * R1 + r] = v; }, c.tw);
    __syncthreads();
    // z inverse stage 2 (radix R2), x V, z forward stage 1 of the (R2, R1) plan: in registers
    {
      constexpr int J = R1;
      constexpr int MAXIT = (N * J + NT - 1) / NT;
      Z<T> v[MAXIT][R2];
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const int it = tid + k * NT;
        if (it < N * J) {
          const int y = it % N, j = it / N;
#pragma unroll
          for (int r = 0; r < R2; ++r) v[k][r] = P[y * LD + j + r * R1];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < MAXIT; ++k) {
        const int it = tid + k * NT;
        if (it < N * J) {
          const int y = it % N, j = it / N;
#pragma unroll
          for (int r = 1; r < R2; ++r) v[k][r] = v[k][r] * twid<+1>(c.tw, r * j);
          dft<R2, +1>(v[k]);
#pragma unroll
          for (int r = 0; r < R2; ++r) {
            const int z = j + r * R1;
            const T w = VL ? VS[y * LD + z] : vg[y * N + z];
            v[k][r] = zscale(v[k][r], w);
          }
          dft<R2, -1>(v[k]);
#pragma unroll
          for (int r = 0; r < R2; ++r) P[y * LD + j * R2 + r] = v[k][r];
        }
      }
    }
    __syncthreads();
    // z forward stage 2 of the (R2, R1) plan: radix R1 over {j + r R2}; keep active z only
    stage<N, R1, -1, true, false, true, NT, N>(
        N, [&](int y, int j, int r) { return P[y * LD + j + r * R2]; },
        [&](int y, int j, int r, Z<T> v) {
          const int z = j + r * R2;
          if (c.zact(z)) P[y * LD + z] = v;
        },
        c.tw);
    __syncthreads();
    y_forward_to_pencils<N, T>(c, tp);
    __syncthreads();  // the next pair overwrites P (and possibly V)
  }
}

// ---- H apply, compact variant: active z lines in LDS, wave-local transforms ----
//
// Per (plane ix, vector) pair only the nza active z lines of the plane are
// kept in LDS, as Q[f][y] (line f of the sphere's z range, all N values of y).
// Each wave owns a contiguous set of those lines for the y transforms, which
// run in place in Q, and a contiguous block of rows y for the z transforms,
// which go through a per-wave scratch of ZR rows x N. Lines and rows never
// cross waves inside a pass, so the stages of a pass need only wave-level
// ordering; a pair needs two workgroup barriers (after the inverse y pass and
// after the z pass). The z transform of a row is inverse stage 1 (radix R1),
// then inverse stage 2 (radix R2), x V_loc and the first stage of the
// reversed forward plan (radix R2) in registers, then forward stage 2 (radix
// R1), keeping the active z only. V_loc is read from a [x][z][y] copy so that
// lanes walking consecutive rows read consecutive addresses.
template <int N, class T, int W, int ZR>
struct PlaneWCfg {
  static constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  static constexpr int RM = R1 > R2 ? R1 : R2;
  // stride of the lines of Q. FP32: the smallest value above N that is 1 mod 32, so that lanes
  // taking consecutive lines (and radix-R1 groups inside a line) fall on different banks. FP64
  // (whose lanes take indices within a line): N + 1, which keeps the LDS of the FP64 kernel at
  // 72^3 within two workgroups per CU.
  static constexpr int QLD = sizeof(T) == 16 ? N + 1 : N + 1 + ((32 - (N + 1) % 32) + 1) % 32;
  static constexpr int NT = 64 * W;
  static constexpr int MAXZ = (ZR * RM + 63) / 64;         // items per lane in a z stage
  // Per-wave z scratch: element (row, l) at row ZR + l plus a skew of ZR per group of R1
  // rows (layout A, written by inverse stage 1) or of R2 rows (layout B, written by the
  // middle stage). The writes of a stage put lanes R1 (or R2) rows apart, which without
  // the skew is a multiple of the bank count; the reads of the next stage take
  // consecutive rows of a group and stay contiguous.
  // Only radices that are powers of two put those lanes a multiple of the bank count apart, and
  // only for them the skew is a shift; other radices keep the plain layout (a division by 9 in
  // the index of every scratch access cost the FP64 pass at 72^3 about a third of its speed).
  static constexpr bool SKEW = (R1 & (R1 - 1)) == 0 && (R2 & (R2 - 1)) == 0;
  static constexpr int SWS = N * ZR + (SKEW ? (N / (R1 < R2 ? R1 : R2)) * ZR : 0);  // elements per wave
  __device__ static constexpr int swa(int row, int l) { return row * ZR + l + (SKEW ? (row / R1) * ZR : 0); }
  __device__ static constexpr int swb(int row, int l) { return row * ZR + l + (SKEW ? (row / R2) * ZR : 0); }
};

// Waves per workgroup and z rows per round of the compact plane kernel. By default
// 4 waves and ZR = 64 / max(R1, R2) rows, so the middle z stage fills the lanes; when
// both radices are multiples of 8 (N = 128: 16 x 8), ZR = 64 / min(R1, R2) fills the
// lanes of the two outer stages as well, with 8 waves to keep two per SIMD, if that
// fits in LDS for the largest set of active z lines a grid of this size can have.
template <int N, class T>
struct PlaneShape {
  static constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  static constexpr int RM = R1 > R2 ? R1 : R2, RMIN = R1 < R2 ? R1 : R2;
  static constexpr int ZR0 = RM >= 64 ? 1 : 64 / RM, ZRW = 64 / RMIN;
  static constexpr int NZA_MAX = 2 * ((N - 1) / 4) + 1;
  static constexpr size_t wide_lds =
      ((size_t)NZA_MAX * PlaneWCfg<N, T, 8, ZRW>::QLD + N + 8 * (size_t)PlaneWCfg<N, T, 8, ZRW>::SWS) * sizeof(Z<T>);
  static constexpr bool wide = R1 % 8 == 0 && R2 % 8 == 0 && RM < 64 && ZRW > ZR0 && wide_lds <= 160 * 1024;
  static constexpr int W = wide ? 8 : 4;
  static constexpr int ZR = wide ? ZRW : ZR0;
};

// Indices [lo, hi] of a y or z transform that no sphere function reaches on any grid
// the basis builds: the grid holds products of two of them (N >= 4 nmax + 1), so the
// active indices [0, nmax] and [N - nmax, N) lie within [0, m] and [N - m, N) for
// m = (N - 1) / 4. Inside unrolled stage loops this is a compile-time constant, and
// the inputs it zeroes and the outputs it drops take no arithmetic.
template <int N>
__device__ constexpr bool idle_range(int lo, int hi) {
  return lo > (N - 1) / 4 && hi < N - (N - 1) / 4;
}

template <int N, class T, int W, int ZR>
constexpr size_t planew_lds_bytes(int nza) {
  return ((size_t)nza * PlaneWCfg<N, T, W, ZR>::QLD + N + (size_t)W * PlaneWCfg<N, T, W, ZR>::SWS) * sizeof(Z<T>);
}

// orders the LDS accesses of one wave: stores above, loads below
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, class T, int W, int ZR, bool PF>
__global__ __launch_bounds__(64 * W) void k_plane_hw(Z<T>* __restrict__ pen, const int* __restrict__ vidx, int nvec,
                                                     const T* __restrict__ vt, FftGeom g) {
  using C = PlaneWCfg<N, T, W, ZR>;
  constexpr int R1 = C::R1, R2 = C::R2, QLD = C::QLD, MAXZ = C::MAXZ;
  extern __shared__ unsigned char smem_raw[];
  const int nza = g.nza, nm = g.zact_lo;
  Z<T>* Q = reinterpret_cast<Z<T>*>(smem_raw);
  Z<T>* tw = Q + (size_t)nza * QLD;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  Z<T>* Sw = tw + N + (size_t)wave * C::SWS;
  {
    const Z<T>* src = twtab<T>(g);
    for (int i = tid; i < N; i += C::NT) tw[i] = src[i];
  }
  __syncthreads();
  const Z<T> zero = zmk(T(0), T(0));
  auto act = [nm](int i) { return i <= nm || i >= N - nm; };             // active y or z index
  auto fz = [nm](int z) { return z <= nm ? z : z - N + 2 * nm + 1; };     // active z -> line
  // this wave's y lines [f0, f0 + nl) and z-pass rows [y0w, y0w + nr)
  const int lpw = (nza + W - 1) / W;
  const int f0 = min(nza, wave * lpw), nl = min(nza, f0 + lpw) - f0;
  // In the y passes that gather from and scatter to the pencils, FP32 lanes take consecutive
  // lines: adjacent pencil columns in HBM and rows QLD apart in LDS (measured on the FP32 pass
  // at 128^3). Items are numbered it = (index within the line) << lsh | (line - f0), with
  // 2^lsh >= nl. FP64 lanes take consecutive indices within a line, it = (line - f0) R + index.
  constexpr bool LINE_FAST = sizeof(T) == 4;
  int lsh = 0;
  while ((1 << lsh) < nl) ++lsh;
  const int lmask = (1 << lsh) - 1;
  // number of items of a gather or scatter pass whose items are transforms of radix R, and
  // the (index, line) of item it (a slot with no line when LINE_FAST pads nl to 2^lsh)
  auto n_items = [&](int R) { return LINE_FAST ? (R << lsh) : nl * R; };
  auto item_ok = [&](int it) { return !LINE_FAST || (it & lmask) < nl; };
  auto item_j = [&](int it, int R) { return LINE_FAST ? (it >> lsh) : it % R; };
  auto item_f = [&](int it, int R) { return f0 + (LINE_FAST ? (it & lmask) : it / R); };
  constexpr int RPW = (N + W - 1) / W;
  const int y0w = min(N, wave * RPW), nr = min(N, y0w + RPW) - y0w;
  const int* __restrict__ yc = g.ycol;
  if (g.live) nvec = min(nvec, *g.live);  // pairs (plane, vector) of the live vectors only
  const long total = (long)N * nvec;
  auto pencils = [&](long q) {
    const int ix = (int)(q / nvec), b = (int)(q - (long)ix * nvec);
    const int vec = vidx ? vidx[b] : b;
    return pen + ((size_t)vec * N + ix) * g.ncol_pad;
  };
  // the first inverse-y item of this lane (it = lane), loaded one pair ahead
  Z<T> pre[R1];
  auto gather = [&](const Z<T>* tp, int it, Z<T>(&v)[R1]) {
    const int j = item_j(it, R2), f = item_f(it, R2);
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int y = j + r * R2;
      v[r] = zero;
      if (!idle_range<N>(r * R2, r * R2 + R2 - 1) && act(y)) {
        const int col = yc[y * nza + f];
        if (col >= 0) v[r] = tp[col];
      }
    }
  };
  const bool lane_item = lane < n_items(R2) && item_ok(lane);  // item it = lane exists
  if (PF && blockIdx.x < total && lane_item) gather(pencils(blockIdx.x), lane, pre);
  for (long q = blockIdx.x; q < total; q += gridDim.x) {
    const int ix = (int)(q / nvec);
    Z<T>* tp = pencils(q);
    const T* __restrict__ vx = vt + (size_t)ix * N * N;
    // ---- inverse y on this wave's lines, in place in Q ----
    for (int it = lane; it < n_items(R2); it += 64) {
      if (!item_ok(it)) continue;
      const int j = item_j(it, R2), f = item_f(it, R2);
      Z<T> v[R1];
      if (PF && it == lane) {
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = pre[r];
      } else {
        gather(tp, it, v);
      }
      dft<R1, +1>(v);
#pragma unroll
      for (int r = 0; r < R1; ++r) Q[f * QLD + j * R1 + r] = v[r];
    }
    wave_sync();
    for (int it = lane; it < nl * R1; it += 64) {
      const int j = it % R1, f = f0 + it / R1;
      Z<T> v[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) v[r] = Q[f * QLD + j + r * R1];
#pragma unroll
      for (int r = 1; r < R2; ++r) v[r] = v[r] * twid<+1>(tw, r * j);
      dft<R2, +1>(v);
#pragma unroll
      for (int r = 0; r < R2; ++r) Q[f * QLD + j + r * R1] = v[r];
    }
    __syncthreads();
    if (PF && q + gridDim.x < total && lane_item) gather(pencils(q + gridDim.x), lane, pre);  // in flight
    // ---- z transforms of this wave's rows, ZR at a time ----
    for (int m0 = 0; m0 < nr; m0 += ZR) {
      const int nz = min(ZR, nr - m0), y0 = y0w + m0;
      // V of this lane's middle-stage item, loaded before the first stage of the round (PF)
      T vreg[MAXZ][R2];
#pragma unroll
      for (int k = 0; k < MAXZ; ++k) {
        const int it = lane + 64 * k;
        const int l = it % ZR, j = it / ZR;
        if (PF && it < ZR * R1 && l < nz) {
#pragma unroll
          for (int r = 0; r < R2; ++r) vreg[k][r] = vx[(size_t)(j + r * R1) * N + y0 + l];
        }
      }
      // inverse stage 1 (radix R1) from the active z of Q
      for (int it = lane; it < ZR * R2; it += 64) {
        const int l = it % ZR, j = it / ZR;
        if (l >= nz) continue;
        Z<T> v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          const int z = j + r * R2;
          v[r] = zero;
          if (!idle_range<N>(r * R2, r * R2 + R2 - 1) && act(z)) v[r] = Q[fz(z) * QLD + y0 + l];
        }
        dft<R1, +1>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) Sw[C::swa(j * R1 + r, l)] = v[r];
      }
      wave_sync();
      // inverse stage 2 (radix R2), x V, forward stage 1 of the reversed plan (radix R2)
      {
        Z<T> v[MAXZ][R2];
#pragma unroll
        for (int k = 0; k < MAXZ; ++k) {
          const int it = lane + 64 * k;
          const int l = it % ZR, j = it / ZR;
          if (it < ZR * R1 && l < nz) {
#pragma unroll
            for (int r = 0; r < R2; ++r) v[k][r] = Sw[C::swa(j + r * R1, l)];
          }
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < MAXZ; ++k) {
          const int it = lane + 64 * k;
          const int l = it % ZR, j = it / ZR;
          if (it < ZR * R1 && l < nz) {
#pragma unroll
            for (int r = 1; r < R2; ++r) v[k][r] = v[k][r] * twid<+1>(tw, r * j);
            dft<R2, +1>(v[k]);
#pragma unroll
            for (int r = 0; r < R2; ++r)
              v[k][r] = zscale(v[k][r], PF ? vreg[k][r] : vx[(size_t)(j + r * R1) * N + y0 + l]);
            dft<R2, -1>(v[k]);
#pragma unroll
            for (int r = 0; r < R2; ++r) Sw[C::swb(j * R2 + r, l)] = v[k][r];
          }
        }
      }
      wave_sync();
      // forward stage 2 (radix R1), active z back into Q
      for (int it = lane; it < ZR * R2; it += 64) {
        const int l = it % ZR, j = it / ZR;
        if (l >= nz) continue;
        Z<T> v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = Sw[C::swb(j + r * R2, l)];
#pragma unroll
        for (int r = 1; r < R1; ++r) v[r] = v[r] * twid<-1>(tw, r * j);
        dft<R1, -1>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          const int z = j + r * R2;
          if (!idle_range<N>(r * R2, r * R2 + R2 - 1) && act(z)) Q[fz(z) * QLD + y0 + l] = v[r];
        }
      }
      wave_sync();
    }
    __syncthreads();
    // ---- forward y on this wave's lines, out to the pencils ----
    // Decimation in frequency, in place in Q: with y = j + R2 r and k = R1 k2 + k1,
    // stage A takes the radix-R1 DFT over r of each j and scales output k1 by
    // w^(j k1); stage B takes the radix-R2 DFT over j of each k1 (a contiguous
    // group) and yields k = R1 k2 + k1.
    for (int it = lane; it < nl * R2; it += 64) {
      const int j = it % R2, f = f0 + it / R2;
      Z<T> v[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) v[r] = Q[f * QLD + j + r * R2];
      dft<R1, -1>(v);
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1) v[k1] = v[k1] * twid<-1>(tw, j * k1);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) Q[f * QLD + j + k1 * R2] = v[k1];
    }
    wave_sync();
    for (int it = lane; it < n_items(R1); it += 64) {
      if (!item_ok(it)) continue;
      const int k1 = item_j(it, R1), f = item_f(it, R1);
      Z<T> v[R2];
#pragma unroll
      for (int jj = 0; jj < R2; ++jj) v[jj] = Q[f * QLD + k1 * R2 + jj];
      dft<R2, -1>(v);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int y = k2 * R1 + k1;
        if (!idle_range<N>(k2 * R1, k2 * R1 + R1 - 1) && act(y)) {
          const int col = yc[y * nza + f];
          if (col >= 0) tp[col] = v[k2];
        }
      }
    }
    wave_sync();  // the next pair's inverse y rewrites this wave's lines of Q
  }
}

// Right-hand sides of one band for every field of a batch: workgroup (ix, bb) keeps
// plane ix of psi_{v0 + bb}(r) in registers (the items of its first stage) and, for
// each field pl, forms psi * dv, transforms the plane and writes the pencils of solve
// pl * nb + bb. psi_v(r) is read once per band instead of once per (band, field).
template <int N>
__global__ __launch_bounds__(plane_nt<N>()) void k_plane_rhs_bands(const Z64* __restrict__ psi_r,
                                                                  const double* __restrict__ dv, int v0, int nb,
                                                                  int i0, int npert, Z64* __restrict__ pen,
                                                                  FftGeom g) {
  using C = PlaneCtx<N, double>;
  constexpr int LD = C::LD, R1 = C::R1, R2 = C::R2, NT = C::NT;
  constexpr int MAXIT = (N * R2 + NT - 1) / NT;
  extern __shared__ unsigned char smem_raw[];
  C c{reinterpret_cast<Z64*>(smem_raw), g.zl, g.ycol, g.nza, g.zact_lo, g.zact_hi,
      plane_twiddles<N, double>(smem_raw, g)};
  Z64* P = c.P;
  const int ix = blockIdx.x, bb = blockIdx.y, tid = threadIdx.x;
  const Z64* __restrict__ ps = psi_r + ((size_t)(v0 + bb) * N + ix) * N * N;
  Z64 pc[MAXIT][R1];
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const int it = tid + k * NT;
    if (it < N * R2) {
      const int y = it / R2, j = it % R2;
#pragma unroll
      for (int r = 0; r < R1; ++r) pc[k][r] = ps[y * N + j + r * R2];
    }
  }
  for (int pl = 0; pl < npert; ++pl) {
    const double* __restrict__ dp = dv + ((size_t)(i0 + pl) * N + ix) * N * N;
    // z forward stage 1 (radix R1 over z = j + R2 r) of the product row
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int it = tid + k * NT;
      if (it < N * R2) {
        const int y = it / R2, j = it % R2;
        Z64 v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) v[r] = zscale(pc[k][r], dp[y * N + j + r * R2]);
        dft<R1, -1>(v);
#pragma unroll
        for (int r = 0; r < R1; ++r) P[y * LD + j * R1 + r] = v[r];
      }
    }
    __syncthreads();
    stage<N, R2, -1, true, false, false, NT, N>(
        N, [&](int y, int j, int r) { return P[y * LD + j + r * R1]; },
        [&](int y, int j, int r, Z64 v) {
          const int z = j + r * R1;
          if (c.zact(z)) P[y * LD + z] = v;
        },
        c.tw);
    __syncthreads();
    y_forward_to_pencils<N, double>(c, pen + ((size_t)(pl * nb + bb) * N + ix) * g.ncol_pad);
    __syncthreads();  // P is rewritten by the next field
  }
}

// inverse yz DFT of the pencils of vector `vec` to the full plane out[vec][ix][iy][iz]
template <int N>
__global__ __launch_bounds__(plane_nt<N>()) void k_plane_full_inv(const Z64* __restrict__ pen, Z64* __restrict__ out,
                                                                 FftGeom g) {
  using C = PlaneCtx<N, double>;
  constexpr int LD = C::LD, R1 = C::R1, R2 = C::R2, NT = C::NT;
  extern __shared__ unsigned char smem_raw[];
  C c{reinterpret_cast<Z64*>(smem_raw), g.zl, g.ycol, g.nza, g.zact_lo, g.zact_hi,
      plane_twiddles<N, double>(smem_raw, g)};
  Z64* P = c.P;
  const int ix = blockIdx.x;
  const int vec = blockIdx.y;
  y_inverse_from_pencils<N, double>(c, pen + ((size_t)vec * N + ix) * g.ncol_pad);
  z_inverse_stage1<N, double>(c);
  Z64* __restrict__ op = out + ((size_t)vec * N + ix) * N * N;
  stage<N, R2, +1, true, false, false, NT, N>(
      N, [&](int y, int j, int r) { return P[y * LD + j + r * R1]; },
      [&](int y, int j, int r, Z64 v) { op[y * N + j + r * R1] = v; }, c.tw);
}

// forward yz DFT of full planes in[vec][ix][iy][iz] -> pencils of vector `vec`
template <int N>
__global__ __launch_bounds__(plane_nt<N>()) void k_plane_full_fwd(const Z64* __restrict__ in, Z64* __restrict__ pen,
                                                                 FftGeom g) {
  using C = PlaneCtx<N, double>;
  constexpr int LD = C::LD, R1 = C::R1, R2 = C::R2, NT = C::NT;
  extern __shared__ unsigned char smem_raw[];
  C c{reinterpret_cast<Z64*>(smem_raw), g.zl, g.ycol, g.nza, g.zact_lo, g.zact_hi,
      plane_twiddles<N, double>(smem_raw, g)};
  Z64* P = c.P;
  const int ix = blockIdx.x;
  const int vec = blockIdx.y;
  const Z64* __restrict__ ip = in + ((size_t)vec * N + ix) * N * N;
  stage<N, R1, -1, false, false, false, NT, N>(
      N, [&](int y, int j, int r) { return ip[y * N + j + r * R2]; },
      [&](int y, int j, int r, Z64 v) { P[y * LD + j * R1 + r] = v; }, c.tw);
  __syncthreads();
  stage<N, R2, -1, true, false, false, NT, N>(
      N, [&](int y, int j, int r) { return P[y * LD + j + r * R1]; },
      [&](int y, int j, int r, Z64 v) {
        const int z = j + r * R1;
        if (c.zact(z)) P[y * LD + z] = v;
      },
      c.tw);
  __syncthreads();
  y_forward_to_pencils<N, double>(c, pen + ((size_t)vec * N + ix) * g.ncol_pad);
}

// One workgroup per (plane ix, perturbation p): for the nb bands of p in band
// order, inverse yz DFT of the solution pencils and accumulation of
// Re conj(psi_v(r)) x(r) in registers (each thread owns the grid points of its
// last-stage items, the same ones for every band).
template <int N>
__global__ __launch_bounds__(plane_nt<N>()) void k_plane_dn(const Z64* __restrict__ pen,
                                                           const Z64* __restrict__ psi_r, int band0, int nb,
                                                           const int* __restrict__ pert_out, double scale,
                                                           double* __restrict__ dn, FftGeom g) {
  using C = PlaneCtx<N, double>;
  constexpr int LD = C::LD, R1 = C::R1, R2 = C::R2, NT = C::NT;
  constexpr int J = R1;
  constexpr int MAXIT = (N * J + NT - 1) / NT;
  extern __shared__ unsigned char smem_raw[];
  C c{reinterpret_cast<Z64*>(smem_raw), g.zl, g.ycol, g.nza, g.zact_lo, g.zact_hi,
      plane_twiddles<N, double>(smem_raw, g)};
  Z64* P = c.P;
  const int ix = blockIdx.x;
  const int pl = blockIdx.y;
  const int tid = threadIdx.x;
  double acc[MAXIT][R2];
#pragma unroll
  for (int k = 0; k < MAXIT; ++k)
#pragma unroll
    for (int r = 0; r < R2; ++r) acc[k][r] = 0.0;
  for (int bb = 0; bb < nb; ++bb) {
    const int s = pl * nb + bb;
    y_inverse_from_pencils<N, double>(c, pen + ((size_t)s * N + ix) * g.ncol_pad);
    z_inverse_stage1<N, double>(c);
    const Z64* __restrict__ ps = psi_r + ((size_t)(band0 + bb) * N + ix) * N * N;
#pragma unroll
    for (int k = 0; k < MAXIT; ++k) {
      const int it = tid + k * NT;
      if (it < N * J) {
        const int y = it / J, j = it - y * J;
        Z64 v[R2];
#pragma unroll
        for (int r = 0; r < R2; ++r) v[r] = P[y * LD + j + r * R1];
#pragma unroll
        for (int r = 1; r < R2; ++r) v[r] = v[r] * twid<+1>(c.tw, r * j);
        dft<R2, +1>(v);
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const Z64 w = ps[y * N + j + r * R1];
          acc[k][r] += w.re * v[r].re + w.im * v[r].im;
        }
      }
    }
    __syncthreads();  // P is rewritten by the next band
  }
  double* __restrict__ dp = dn + ((size_t)pert_out[pl] * N + ix) * N * N;
#pragma unroll
  for (int k = 0; k < MAXIT; ++k) {
    const int it = tid + k * NT;
    if (it < N * J) {
      const int y = it / J, j = it - y * J;
#pragma unroll
      for (int r = 0; r < R2; ++r) dp[y * N + j + r * R1] = scale * acc[k][r];
    }
  }
}

// ---- FP64 full-plane transforms for grids whose plane does not fit in LDS ----
//
// The right-hand side, psi_v(r) and dn kernels above hold a whole N x N plane
// in LDS. For the larger grids (108, 128) they run in the compact layout of
// the H-apply kernel instead: only the nza active z lines of the plane sit in
// LDS (Q[f][y]), the y transforms run wave-locally on them, and each wave
// takes its block of rows y through the z transform ZR rows at a time via its
// own scratch, reading or writing the full-grid row directly in HBM.

// inverse y of this wave's active lines [f0, f0 + nl) from the pencils tp
template <int N>
__device__ __forceinline__ void cw_y_inverse(Z64* __restrict__ Q, const Z64* __restrict__ tw, const Z64* __restrict__ tp,
                                             const int* __restrict__ yc, int nza, int nm, int f0, int nl, int lane) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2, QLD = N + 1;
  const Z64 zero = zmk(0.0, 0.0);
  for (int it = lane; it < nl * R2; it += 64) {
    const int j = it % R2, f = f0 + it / R2;
    Z64 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int y = j + r * R2;
      v[r] = zero;
      if (y <= nm || y >= N - nm) {
        const int col = yc[y * nza + f];
        if (col >= 0) v[r] = tp[col];
      }
    }
    dft<R1, +1>(v);
#pragma unroll
    for (int r = 0; r < R1; ++r) Q[f * QLD + j * R1 + r] = v[r];
  }
  wave_sync();
  for (int it = lane; it < nl * R1; it += 64) {
    const int j = it % R1, f = f0 + it / R1;
    Z64 v[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) v[r] = Q[f * QLD + j + r * R1];
#pragma unroll
    for (int r = 1; r < R2; ++r) v[r] = v[r] * twid<+1>(tw, r * j);
    dft<R2, +1>(v);
#pragma unroll
    for (int r = 0; r < R2; ++r) Q[f * QLD + j + r * R1] = v[r];
  }
}

// forward y of this wave's active lines to the pencils tp (decimation in frequency, in place)
template <int N>
__device__ __forceinline__ void cw_y_forward(Z64* __restrict__ Q, const Z64* __restrict__ tw, Z64* __restrict__ tp,
                                             const int* __restrict__ yc, int nza, int nm, int f0, int nl, int lane) {
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2, QLD = N + 1;
  for (int it = lane; it < nl * R2; it += 64) {
    const int j = it % R2, f = f0 + it / R2;
    Z64 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) v[r] = Q[f * QLD + j + r * R2];
    dft<R1, -1>(v);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) v[k1] = v[k1] * twid<-1>(tw, j * k1);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) Q[f * QLD + j + k1 * R2] = v[k1];
  }
  wave_sync();
  for (int it = lane; it < nl * R1; it += 64) {
    const int k1 = it % R1, f = f0 + it / R1;
    Z64 v[R2];
#pragma unroll
    for (int jj = 0; jj < R2; ++jj) v[jj] = Q[f * QLD + k1 * R2 + jj];
    dft<R2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      const int y = k2 * R1 + k1;
      if (y <= nm || y >= N - nm) {
        const int col = yc[y * nza + f];
        if (col >= 0) tp[col] = v[k2];
      }
    }
  }
}

template <int N>
struct CwCfg {
  static constexpr int W = 4;
  static constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  static constexpr int RM = R1 > R2 ? R1 : R2;
  static constexpr int ZR = RM >= 64 ? 1 : 64 / RM;
  static constexpr int RPW = (N + W - 1) / W;               // rows y per wave
  static constexpr int RND = (RPW + ZR - 1) / ZR;           // z rounds per wave
  static constexpr int MAXZ = (ZR * RM + 63) / 64;          // items per lane in a z stage
};

// shared set-up: LDS carve-out, twiddles, this wave's lines and rows
#define STERN_CW_SETUP                                                          \
  using C = CwCfg<N>;                                                           \
  constexpr int R1 = C::R1, R2 = C::R2, ZR = C::ZR, QLD = N + 1;                \
  extern __shared__ unsigned char smem_raw[];                                   \
  const int nza = g.nza, nm = g.zact_lo;                                        \
  Z64* Q = reinterpret_cast<Z64*>(smem_raw);                                    \
  Z64* tw = Q + (size_t)nza * QLD;                                              \
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;                \
  Z64* Sw = tw + N + (size_t)wave * N * ZR;                                     \
  for (int i = tid; i < N; i += 64 * C::W) tw[i] = g.tw64[i];                   \
  const int lpw = (nza + C::W - 1) / C::W;                                      \
  const int f0 = min(nza, wave * lpw), nl = min(nza, f0 + lpw) - f0;            \
  const int y0w = min(N, wave * C::RPW), nr = min(N, y0w + C::RPW) - y0w;       \
  (void)nr;                                                                     \
  auto act = [nm](int i) { return i <= nm || i >= N - nm; };                    \
  auto fz = [nm](int z) { return z <= nm ? z : z - N + 2 * nm + 1; };           \
  (void)act;                                                                    \
  (void)fz;                                                                     \
  __syncthreads();

// right-hand side: pencils[s] of plane ix = forward yz DFT of psi_r[band[s]] * dv[pert[s]]
template <int N>
__global__ __launch_bounds__(256) void k_plane_rhs_c(const Z64* __restrict__ psi_r, const double* __restrict__ dv,
                                                    const int* __restrict__ band, const int* __restrict__ pert,
                                                    Z64* __restrict__ pen, FftGeom g) {
  STERN_CW_SETUP
  const int ix = blockIdx.x, s = blockIdx.y;
  const Z64* __restrict__ ps = psi_r + ((size_t)band[s] * N + ix) * N * N;
  const double* __restrict__ dp = dv + ((size_t)pert[s] * N + ix) * N * N;
  for (int m0 = 0; m0 < nr; m0 += ZR) {
    const int nz = min(ZR, nr - m0), y0 = y0w + m0;
    // forward stage 1 (radix R2) over z = j + R1 r of the product row
#pragma unroll
    for (int k = 0; k < C::MAXZ; ++k) {
      const int it = lane + 64 * k;
      if (it < nz * R1) {
        const int l = it % nz, j = it / nz;
        const size_t row = (size_t)(y0 + l) * N;
        Z64 v[R2];
#pragma unroll
        for (int r = 0; r < R2; ++r) v[r] = zscale(ps[row + j + r * R1], dp[row + j + r * R1]);
        dft<R2, -1>(v);
#pragma unroll
        for (int r = 0; r < R2; ++r) Sw[(j * R2 + r) * ZR + l] = v[r];
      }
    }
    wave_sync();
    // forward stage 2 (radix R1), active z into Q
    for (int it = lane; it < nz * R2; it += 64) {
      const int l = it % nz, j = it / nz;
      Z64 v[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) v[r] = Sw[(j + r * R2) * ZR + l];
#pragma unroll
      for (int r = 1; r < R1; ++r) v[r] = v[r] * twid<-1>(tw, r * j);
      dft<R1, -1>(v);
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int z = j + r * R2;
        if (act(z)) Q[fz(z) * QLD + y0 + l] = v[r];
      }
    }
    wave_sync();
  }
  __syncthreads();
  cw_y_forward<N>(Q, tw, pen + ((size_t)s * N + ix) * g.ncol_pad, g.ycol, nza, nm, f0, nl, lane);
}

// inverse z of one round of this wave's rows, from the active lines in Q; calls
// emit(k, l, j, v) with v[r] the value at row y0 + l, z = j + R1 r
template <int N, class Emit>
__device__ __forceinline__ void cw_z_inverse_round(const Z64* __restrict__ Q, const Z64* __restrict__ tw,
                                                   Z64* __restrict__ Sw, int nm, int y0, int nz, int lane,
                                                   Emit&& emit) {
  using C = CwCfg<N>;
  constexpr int R1 = C::R1, R2 = C::R2, ZR = C::ZR, QLD = N + 1;
  const Z64 zero = zmk(0.0, 0.0);
  for (int it = lane; it < nz * R2; it += 64) {
    const int l = it % nz, j = it / nz;
    Z64 v[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int z = j + r * R2;
      v[r] = zero;
      if (z <= nm || z >= N - nm) v[r] = Q[(z <= nm ? z : z - N + 2 * nm + 1) * QLD + y0 + l];
    }
    dft<R1, +1>(v);
#pragma unroll
    for (int r = 0; r < R1; ++r) Sw[(j * R1 + r) * ZR + l] = v[r];
  }
  wave_sync();
#pragma unroll
  for (int k = 0; k < C::MAXZ; ++k) {
    const int it = lane + 64 * k;
    if (it < nz * R1) {
      const int l = it % nz, j = it / nz;
      Z64 v[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) v[r] = Sw[(j + r * R1) * ZR + l];
#pragma unroll
      for (int r = 1; r < R2; ++r) v[r] = v[r] * twid<+1>(tw, r * j);
      dft<R2, +1>(v);
      emit(k, l, j, v);
    }
  }
  wave_sync();  // the next round rewrites Sw
}

// inverse yz DFT of the pencils of vector `vec` to the full plane out[vec][ix][iy][iz]
template <int N>
__global__ __launch_bounds__(256) void k_plane_full_inv_c(const Z64* __restrict__ pen, Z64* __restrict__ out,
                                                         FftGeom g) {
  STERN_CW_SETUP
  const int ix = blockIdx.x, vec = blockIdx.y;
  cw_y_inverse<N>(Q, tw, pen + ((size_t)vec * N + ix) * g.ncol_pad, g.ycol, nza, nm, f0, nl, lane);
  __syncthreads();
  Z64* __restrict__ op = out + ((size_t)vec * N + ix) * N * N;
  for (int m0 = 0; m0 < nr; m0 += ZR) {
    const int y0 = y0w + m0;
    cw_z_inverse_round<N>(Q, tw, Sw, nm, y0, min(ZR, nr - m0), lane, [&](int, int l, int j, const Z64(&v)[R2]) {
#pragma unroll
      for (int r = 0; r < R2; ++r) op[(size_t)(y0 + l) * N + j + r * R1] = v[r];
    });
  }
}

// dn of perturbation pl over nb bands: as k_plane_dn, with each wave's rows
// accumulated in registers across the bands (RND rounds x MAXZ items x R2 values)
template <int N>
__global__ __launch_bounds__(256) void k_plane_dn_c(const Z64* __restrict__ pen, const Z64* __restrict__ psi_r,
                                                   int band0, int nb, const int* __restrict__ pert_out, double scale,
                                                   double* __restrict__ dn, FftGeom g) {
  STERN_CW_SETUP
  const int ix = blockIdx.x, pl = blockIdx.y;
  double acc[C::RND][C::MAXZ][R2];
#pragma unroll
  for (int m = 0; m < C::RND; ++m)
#pragma unroll
    for (int k = 0; k < C::MAXZ; ++k)
#pragma unroll
      for (int r = 0; r < R2; ++r) acc[m][k][r] = 0.0;
  for (int bb = 0; bb < nb; ++bb) {
    const int s = pl * nb + bb;
    cw_y_inverse<N>(Q, tw, pen + ((size_t)s * N + ix) * g.ncol_pad, g.ycol, nza, nm, f0, nl, lane);
    __syncthreads();
    const Z64* __restrict__ ps = psi_r + ((size_t)(band0 + bb) * N + ix) * N * N;
#pragma unroll
    for (int m = 0; m < C::RND; ++m) {
      const int m0 = m * ZR;
      if (m0 < nr) {
        const int y0 = y0w + m0;
        cw_z_inverse_round<N>(Q, tw, Sw, nm, y0, min(ZR, nr - m0), lane, [&](int k, int l, int j, const Z64(&v)[R2]) {
#pragma unroll
          for (int r = 0; r < R2; ++r) {
            const Z64 w = ps[(size_t)(y0 + l) * N + j + r * R1];
            acc[m][k][r] += w.re * v[r].re + w.im * v[r].im;
          }
        });
      }
    }
    __syncthreads();  // Q is rewritten by the next band
  }
  double* __restrict__ dp = dn + ((size_t)pert_out[pl] * N + ix) * N * N;
#pragma unroll
  for (int m = 0; m < C::RND; ++m) {
    const int m0 = m * ZR;
    if (m0 < nr) {
      const int nz = min(ZR, nr - m0), y0 = y0w + m0;
#pragma unroll
      for (int k = 0; k < C::MAXZ; ++k) {
        const int it = lane + 64 * k;
        if (it < nz * R1) {
          const int l = it % nz, j = it / nz;
#pragma unroll
          for (int r = 0; r < R2; ++r) dp[(size_t)(y0 + l) * N + j + r * R1] = scale * acc[m][k][r];
        }
      }
    }
  }
}
#undef STERN_CW_SETUP

// Raise the dynamic LDS limit of a plane kernel once per instantiation
// (thread-safe: several host threads may launch concurrently).
void set_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static const void* done[256];
  static int ndone = 0;
  if (bytes <= 64 * 1024) return;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < ndone; ++i)
    if (done[i] == kernel) return;
  (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (ndone < 256) done[ndone++] = kernel;
}

}  // namespace

bool fft_size_supported(int N) {
  switch (N) {
    case 8: case 9: case 12: case 16: case 18: case 24: case 27: case 32: case 36:
    case 48: case 54: case 64: case 72: case 81: case 96: case 108: case 128:
      return true;
    default:
      return false;
  }
}

size_t plane_lds_bytes(int N, int elem_bytes) { return ((size_t)N * (N + 1) + N) * elem_bytes; }

#define STERN_DISPATCH_N(N_, CALL)                     \
  switch (N_) {                                        \
    case 8: { constexpr int NN = 8; CALL; } break;     \
    case 9: { constexpr int NN = 9; CALL; } break;     \
    case 12: { constexpr int NN = 12; CALL; } break;   \
    case 16: { constexpr int NN = 16; CALL; } break;   \
    case 18: { constexpr int NN = 18; CALL; } break;   \
    case 24: { constexpr int NN = 24; CALL; } break;   \
    case 27: { constexpr int NN = 27; CALL; } break;   \
    case 32: { constexpr int NN = 32; CALL; } break;   \
    case 36: { constexpr int NN = 36; CALL; } break;   \
    case 48: { constexpr int NN = 48; CALL; } break;   \
    case 54: { constexpr int NN = 54; CALL; } break;   \
    case 64: { constexpr int NN = 64; CALL; } break;   \
    case 72: { constexpr int NN = 72; CALL; } break;   \
    case 81: { constexpr int NN = 81; CALL; } break;   \
    case 96: { constexpr int NN = 96; CALL; } break;   \
    case 108: { constexpr int NN = 108; CALL; } break; \
    case 128: { constexpr int NN = 128; CALL; } break; \
    default: break;                                    \
  }

template <class T>
void launch_xinv(const FftGeom& g, const Z<T>* sph, const int* vidx, int nvec, Z<T>* pen, hipStream_t st) {
  if (nvec <= 0) return;
  dim3 grid(g.ncol_pad / col_block<T>(), nvec);
  STERN_DISPATCH_N(g.N, (k_xinv<NN, T><<<grid, kXThreads, 0, st>>>(sph, vidx, pen, g)));
}
template void launch_xinv<double>(const FftGeom&, const Z64*, const int*, int, Z64*, hipStream_t);
template void launch_xinv<float>(const FftGeom&, const Z32*, const int*, int, Z32*, hipStream_t);

template <class T>
void launch_xfwd(const FftGeom& g, const Z<T>* pen, const int* vidx, int nvec, Z<T>* out, int mode, const Z<T>* pin,
                 const double* eps, double scale, hipStream_t st) {
  if (nvec <= 0) return;
  dim3 grid(g.ncol_pad / col_block<T>(), nvec);
  if (mode == 0) {
    STERN_DISPATCH_N(g.N, (k_xfwd<NN, T, 0><<<grid, kXThreads, 0, st>>>(pen, vidx, out, pin, eps, scale, g)));
  } else if (mode == 1) {
    STERN_DISPATCH_N(g.N, (k_xfwd<NN, T, 1><<<grid, kXThreads, 0, st>>>(pen, vidx, out, pin, eps, scale, g)));
  } else {
    STERN_DISPATCH_N(g.N, (k_xfwd<NN, T, 2><<<grid, kXThreads, 0, st>>>(pen, vidx, out, pin, eps, scale, g)));
  }
}
template void launch_xfwd<double>(const FftGeom&, const Z64*, const int*, int, Z64*, int, const Z64*, const double*,
                                  double, hipStream_t);
template void launch_xfwd<float>(const FftGeom&, const Z32*, const int*, int, Z32*, int, const Z32*, const double*,
                                 double, hipStream_t);

template <class T>
void launch_plane_vloc(const FftGeom& g, Z<T>* pen, const int* vidx, int nvec, const T* v_r, hipStream_t st) {
  if (nvec <= 0) return;
  STERN_DISPATCH_N(g.N, ({
                     const size_t lds = vloc_lds_bytes<NN, T>(vloc_v_in_lds<NN, T>());
                     set_lds((const void*)k_plane_vloc<NN, T>, lds);
                     const int per_cu = lds > 80 * 1024 ? 1 : (lds > 53 * 1024 ? 2 : 3);
                     const long pairs = (long)NN * nvec;
                     const int grid = (int)std::min<long>(pairs, (long)g.n_cu * per_cu);
                     k_plane_vloc<NN, T><<<grid, plane_nt<NN, T>(), lds, st>>>(pen, vidx, nvec, v_r, g);
                   }));
}
template void launch_plane_vloc<double>(const FftGeom&, Z64*, const int*, int, const double*, hipStream_t);
namespace {
// resident workgroups per CU of a kernel at a block size and dynamic LDS size (cached)
int blocks_per_cu(const void* kernel, int nt, size_t lds) {
  static std::mutex mu;
  struct E {
    const void* k;
    int nt;
    size_t lds;
    int n;
  };
  static E cache[256];
  static int nc = 0;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < nc; ++i)
    if (cache[i].k == kernel && cache[i].nt == nt && cache[i].lds == lds) return cache[i].n;
  if (lds > 64 * 1024) (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, nt, lds) != hipSuccess || n < 1) n = 1;
  if (nc < 256) cache[nc++] = E{kernel, nt, lds, n};
  return n;
}
}  // namespace

template <int NN, class T, bool PF>
void launch_plane_hw_n(const FftGeom& g, Z<T>* pen, const int* vidx, int nvec, const T* vt, hipStream_t st) {
  constexpr int W = PlaneShape<NN, T>::W, ZR = PlaneShape<NN, T>::ZR;
  const size_t lds = planew_lds_bytes<NN, T, W, ZR>(g.nza);
  const void* kp = (const void*)k_plane_hw<NN, T, W, ZR, PF>;
  const int per_cu = blocks_per_cu(kp, 64 * W, lds);
  const long pairs = (long)NN * nvec;
  const int grid = (int)std::min<long>(pairs, (long)g.n_cu * per_cu);
  k_plane_hw<NN, T, W, ZR, PF><<<grid, 64 * W, lds, st>>>(pen, vidx, nvec, vt, g);
}

// prefetch: also load the next pair's first inverse-y items and each round's V
// ahead of use (more registers, fewer exposed load latencies)
template <class T>
void launch_plane_hw(const FftGeom& g, Z<T>* pen, const int* vidx, int nvec, const T* vt, bool prefetch,
                     hipStream_t st) {
  if (nvec <= 0) return;
  STERN_DISPATCH_N(g.N, ({
                     if (prefetch)
                       launch_plane_hw_n<NN, T, true>(g, pen, vidx, nvec, vt, st);
                     else
                       launch_plane_hw_n<NN, T, false>(g, pen, vidx, nvec, vt, st);
                   }));
}
size_t plane_hw_lds(int N, int nza, bool fp64) {
  size_t r = 0;
  STERN_DISPATCH_N(N, ({
                     using S64 = PlaneShape<NN, double>;
                     using S32 = PlaneShape<NN, float>;
                     r = fp64 ? planew_lds_bytes<NN, double, S64::W, S64::ZR>(nza)
                              : planew_lds_bytes<NN, float, S32::W, S32::ZR>(nza);
                   }));
  return r;
}
template void launch_plane_hw<double>(const FftGeom&, Z64*, const int*, int, const double*, bool, hipStream_t);
template void launch_plane_hw<float>(const FftGeom&, Z32*, const int*, int, const float*, bool, hipStream_t);

template void launch_plane_vloc<float>(const FftGeom&, Z32*, const int*, int, const float*, hipStream_t);

// FP64 full-plane kernels hold the whole plane when it fits in LDS, else the compact layout
template <int N>
constexpr bool full_plane_fits() {
  return ((size_t)N * (N + 1) + N) * sizeof(Z64) <= 160 * 1024;
}
template <int N>
size_t cw_lds_bytes(int nza) {
  return ((size_t)nza * (N + 1) + N + (size_t)CwCfg<N>::W * N * CwCfg<N>::ZR) * sizeof(Z64);
}

void launch_plane_rhs(const FftGeom& g, const Z64* psi_r, const double* dv, int v0, int nb, int i0, int npert,
                      const int* band, const int* pert, Z64* pen, hipStream_t st) {
  if (nb <= 0 || npert <= 0) return;
  STERN_DISPATCH_N(g.N, ({
                     if constexpr (full_plane_fits<NN>()) {
                       const size_t lds = plane_lds_bytes(NN, sizeof(Z64));
                       set_lds((const void*)k_plane_rhs_bands<NN>, lds);
                       k_plane_rhs_bands<NN><<<dim3(NN, nb), plane_nt<NN>(), lds, st>>>(psi_r, dv, v0, nb, i0,
                                                                                      npert, pen, g);
                     } else {
                       const size_t lds = cw_lds_bytes<NN>(g.nza);
                       set_lds((const void*)k_plane_rhs_c<NN>, lds);
                       k_plane_rhs_c<NN><<<dim3(NN, nb * npert), 256, lds, st>>>(psi_r, dv, band, pert, pen, g);
                     }
                   }));
}

void launch_plane_full_inv(const FftGeom& g, const Z64* pen, int nvec, Z64* out, hipStream_t st) {
  if (nvec <= 0) return;
  dim3 grid(g.N, nvec);
  STERN_DISPATCH_N(g.N, ({
                     if constexpr (full_plane_fits<NN>()) {
                       const size_t lds = plane_lds_bytes(NN, sizeof(Z64));
                       set_lds((const void*)k_plane_full_inv<NN>, lds);
                       k_plane_full_inv<NN><<<grid, plane_nt<NN>(), lds, st>>>(pen, out, g);
                     } else {
                       const size_t lds = cw_lds_bytes<NN>(g.nza);
                       set_lds((const void*)k_plane_full_inv_c<NN>, lds);
                       k_plane_full_inv_c<NN><<<grid, 256, lds, st>>>(pen, out, g);
                     }
                   }));
}

bool plane_full_fwd_fits(int N, size_t lds) { return plane_lds_bytes(N, sizeof(Z64)) <= lds; }

void launch_plane_full_fwd(const FftGeom& g, const Z64* in, int nvec, Z64* pen, hipStream_t st) {
  if (nvec <= 0) return;
  const size_t lds = plane_lds_bytes(g.N, sizeof(Z64));
  dim3 grid(g.N, nvec);
  STERN_DISPATCH_N(g.N, (set_lds((const void*)k_plane_full_fwd<NN>, lds),
                         k_plane_full_fwd<NN><<<grid, plane_nt<NN>(), lds, st>>>(in, pen, g)));
}

void launch_plane_dn(const FftGeom& g, const Z64* pen, const Z64* psi_r, int band0, int nb, int npert,
                     const int* pert_out, double scale, double* dn, hipStream_t st) {
  if (npert <= 0 || nb <= 0) return;
  dim3 grid(g.N, npert);
  STERN_DISPATCH_N(g.N, ({
                     if constexpr (full_plane_fits<NN>()) {
                       const size_t lds = plane_lds_bytes(NN, sizeof(Z64));
                       set_lds((const void*)k_plane_dn<NN>, lds);
                       k_plane_dn<NN><<<grid, plane_nt<NN>(), lds, st>>>(pen, psi_r, band0, nb, pert_out, scale,
                                                                        dn, g);
                     } else {
                       const size_t lds = cw_lds_bytes<NN>(g.nza);
                       set_lds((const void*)k_plane_dn_c<NN>, lds);
                       k_plane_dn_c<NN><<<grid, 256, lds, st>>>(pen, psi_r, band0, nb, pert_out, scale, dn, g);
                     }
                   }));
}

// LDS of the FP64 plane kernels of the RHS, psi_v(r) and dn for grid N
size_t plane_fp64_lds(int N, int nza) {
  size_t r = 0;
  STERN_DISPATCH_N(N, ({
                     if constexpr (full_plane_fits<NN>())
                       r = plane_lds_bytes(NN, sizeof(Z64));
                     else
                       r = cw_lds_bytes<NN>(nza);
                   }));
  return r;
}

}  // namespace stern
