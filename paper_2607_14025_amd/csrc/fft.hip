// Pruned 3-D FFT kernels of the H apply, the right-hand side and the density
// response, FP64. A vector on the plane-wave sphere goes through
//   x pass:  per x-pencil column (n_y, n_z) of the sphere, length-N DFT along x
//   yz pass: per plane ix, 2-D DFT over the columns' (iy, iz) positions
// so only the sphere's columns are ever read from or written to HBM.
#include "fft_dev.hpp"
#include "kernels.hpp"

namespace stern {

namespace {

template <int N>
constexpr int plane_threads() {
  return N >= 48 ? 512 : 256;
}
constexpr int kXThreads = 128;

// ---------------------------------------------------------------- x pass ----
template <int N>
__global__ __launch_bounds__(kXThreads) void k_xinv(const Z64* __restrict__ sph, const int* __restrict__ vidx,
                                                    Z64* __restrict__ pen, FftGeom g) {
  constexpr int CB = kColBlock, LDX = N + 1;
  __shared__ Z64 P[CB * LDX];
  const int c0 = blockIdx.x * CB;
  const int vec = vidx ? vidx[blockIdx.y] : blockIdx.y;
  for (int i = threadIdx.x; i < CB * LDX; i += kXThreads) P[i] = zmk(0.0, 0.0);
  __syncthreads();
  const Z64* src = sph + (size_t)vec * g.npw_pad;
  for (int i = threadIdx.x; i < CB * N; i += kXThreads) {
    const int cc = i / N, t = i - cc * N;
    const int c = c0 + cc;
    if (t < g.col_len[c]) {
      int nx = g.col_xmin[c] + t;
      nx += (nx < 0) ? N : 0;
      P[cc * LDX + nx] = src[g.col_start[c] + t];
    }
  }
  __syncthreads();
  fft_lines<N, +1, kXThreads, CB>(P, CB, 1, [](int f) { return f * LDX; }, NoPost{}, g.tw64);
  Z64* dst = pen + (size_t)vec * N * g.ncol_pad + c0;
  for (int i = threadIdx.x; i < CB * N; i += kXThreads) {
    const int ix = i / CB, cc = i - ix * CB;
    dst[(size_t)ix * g.ncol_pad + cc] = P[cc * LDX + ix];
  }
}

template <int N, int MODE>
__global__ __launch_bounds__(kXThreads) void k_xfwd(const Z64* __restrict__ pen, const int* __restrict__ vidx,
                                                    Z64* __restrict__ out, const Z64* __restrict__ pin,
                                                    const double* __restrict__ eps, double scale, FftGeom g) {
  constexpr int CB = kColBlock, LDX = N + 1;
  __shared__ Z64 P[CB * LDX];
  const int c0 = blockIdx.x * CB;
  const int vec = vidx ? vidx[blockIdx.y] : blockIdx.y;
  const Z64* src = pen + (size_t)vec * N * g.ncol_pad + c0;
  for (int i = threadIdx.x; i < CB * N; i += kXThreads) {
    const int ix = i / CB, cc = i - ix * CB;
    P[cc * LDX + ix] = src[(size_t)ix * g.ncol_pad + cc];
  }
  __syncthreads();
  fft_lines<N, -1, kXThreads, CB>(P, CB, 1, [](int f) { return f * LDX; }, NoPost{}, g.tw64);
  Z64* dst = out + (size_t)vec * g.npw_pad;
  const Z64* pv = (MODE == 1) ? pin + (size_t)vec * g.npw_pad : nullptr;
  const double e = (MODE == 1) ? eps[vec] : 0.0;
  for (int i = threadIdx.x; i < CB * N; i += kXThreads) {
    const int cc = i / N, t = i - cc * N;
    const int c = c0 + cc;
    if (t < g.col_len[c]) {
      int nx = g.col_xmin[c] + t;
      nx += (nx < 0) ? N : 0;
      const int gi = g.col_start[c] + t;
      Z64 v = P[cc * LDX + nx];
      if (MODE == 1) {
        const double d = g.g2h[gi] - e;
        const Z64 pp = pv[gi];
        v = zmk(v.re + d * pp.re, v.im + d * pp.im);
      } else if (MODE == 2) {
        v = zscale(v, scale);
      }
      dst[gi] = v;
    }
  }
}

// --------------------------------------------------------------- yz pass ----
template <int N>
__device__ __forceinline__ void plane_scatter(Z64* P, const Z64* __restrict__ src, const FftGeom& g, int NT) {
  constexpr int LD = N + 1;
  for (int c = threadIdx.x; c < g.ncol; c += NT) {
    const int p = g.col_pos[c];
    const int iy = p / N, iz = p - iy * N;
    P[iy * LD + iz] = src[c];
  }
}

template <int N>
__device__ __forceinline__ void plane_zero(Z64* P, int NT) {
  constexpr int LD = N + 1;
  for (int i = threadIdx.x; i < N * LD; i += NT) P[i] = zmk(0.0, 0.0);
}

template <int N>
__global__ __launch_bounds__(plane_threads<N>()) void k_plane_vloc(Z64* __restrict__ pen, const int* __restrict__ vidx,
                                                                  const double* __restrict__ v_r, FftGeom g) {
  constexpr int NT = plane_threads<N>(), LD = N + 1;
  extern __shared__ unsigned char smem_raw[];
  Z64* P = reinterpret_cast<Z64*>(smem_raw);
  const int ix = blockIdx.x;
  const int vec = vidx ? vidx[blockIdx.y] : blockIdx.y;
  Z64* tp = pen + ((size_t)vec * N + ix) * g.ncol_pad;
  plane_zero<N>(P, NT);
  __syncthreads();
  plane_scatter<N>(P, tp, g, NT);
  __syncthreads();
  const int* zl = g.zl;
  auto zline = [zl](int f) { return zl[f]; };
  auto row = [](int f) { return f * LD; };
  fft_lines<N, +1, NT, N>(P, g.nza, LD, zline, NoPost{}, g.tw64);
  const double* vp = v_r + (size_t)ix * N * N;
  fft_lines<N, +1, NT, N>(
      P, N, 1, row, [vp](int f, int n, int, int, Z64 v) { return zscale(v, vp[f * N + n]); }, g.tw64);
  fft_lines<N, -1, NT, N>(P, N, 1, row, NoPost{}, g.tw64);
  fft_lines<N, -1, NT, N>(P, g.nza, LD, zline, NoPost{}, g.tw64);
  for (int c = threadIdx.x; c < g.ncol; c += NT) {
    const int p = g.col_pos[c];
    const int iy = p / N, iz = p - iy * N;
    tp[c] = P[iy * LD + iz];
  }
}

template <int N>
__global__ __launch_bounds__(plane_threads<N>()) void k_plane_rhs(const Z64* __restrict__ psi_r,
                                                                 const double* __restrict__ dv,
                                                                 const int* __restrict__ band,
                                                                 const int* __restrict__ pert,
                                                                 Z64* __restrict__ pen, FftGeom g) {
  constexpr int NT = plane_threads<N>(), LD = N + 1;
  extern __shared__ unsigned char smem_raw[];
  Z64* P = reinterpret_cast<Z64*>(smem_raw);
  const int ix = blockIdx.x;
  const int s = blockIdx.y;
  const Z64* ps = psi_r + ((size_t)band[s] * N + ix) * N * N;
  const double* dp = dv + ((size_t)pert[s] * N + ix) * N * N;
  for (int i = threadIdx.x; i < N * N; i += NT) {
    const int iy = i / N, iz = i - iy * N;
    P[iy * LD + iz] = zscale(ps[i], dp[i]);
  }
  __syncthreads();
  auto row = [](int f) { return f * LD; };
  const int* zl = g.zl;
  fft_lines<N, -1, NT, N>(P, N, 1, row, NoPost{}, g.tw64);
  fft_lines<N, -1, NT, N>(P, g.nza, LD, [zl](int f) { return zl[f]; }, NoPost{}, g.tw64);
  Z64* tp = pen + ((size_t)s * N + ix) * g.ncol_pad;
  for (int c = threadIdx.x; c < g.ncol; c += NT) {
    const int p = g.col_pos[c];
    const int iy = p / N, iz = p - iy * N;
    tp[c] = P[iy * LD + iz];
  }
}

template <int N>
__global__ __launch_bounds__(plane_threads<N>()) void k_plane_full_inv(const Z64* __restrict__ pen,
                                                                      Z64* __restrict__ out, FftGeom g) {
  constexpr int NT = plane_threads<N>(), LD = N + 1;
  extern __shared__ unsigned char smem_raw[];
  Z64* P = reinterpret_cast<Z64*>(smem_raw);
  const int ix = blockIdx.x;
  const int vec = blockIdx.y;
  plane_zero<N>(P, NT);
  __syncthreads();
  plane_scatter<N>(P, pen + ((size_t)vec * N + ix) * g.ncol_pad, g, NT);
  __syncthreads();
  const int* zl = g.zl;
  fft_lines<N, +1, NT, N>(P, g.nza, LD, [zl](int f) { return zl[f]; }, NoPost{}, g.tw64);
  fft_lines<N, +1, NT, N>(P, N, 1, [](int f) { return f * LD; }, NoPost{}, g.tw64);
  Z64* op = out + ((size_t)vec * N + ix) * N * N;
  for (int i = threadIdx.x; i < N * N; i += NT) {
    const int iy = i / N, iz = i - iy * N;
    op[i] = P[iy * LD + iz];
  }
}

// One workgroup per (plane ix, perturbation p): accumulates the nb bands of the
// perturbation in band order, each thread keeping the grid points it owns in
// the last FFT stage in registers.
template <int N>
__global__ __launch_bounds__(plane_threads<N>()) void k_plane_dn(const Z64* __restrict__ pen,
                                                                const Z64* __restrict__ psi_r, int band0, int nb,
                                                                const int* __restrict__ pert_out, double scale,
                                                                double* __restrict__ dn, FftGeom g) {
  constexpr int NT = plane_threads<N>(), LD = N + 1;
  constexpr int R1 = Plan<N>::R1, R2 = Plan<N>::R2;
  constexpr int NSLOT = (R2 == 1) ? (N + NT - 1) / NT : (N * R1 + NT - 1) / NT;
  constexpr int NR = (R2 == 1) ? R1 : R2;
  extern __shared__ unsigned char smem_raw[];
  Z64* P = reinterpret_cast<Z64*>(smem_raw);
  const int ix = blockIdx.x;
  const int pl = blockIdx.y;
  double acc[NSLOT][NR];
#pragma unroll
  for (int a = 0; a < NSLOT; ++a)
#pragma unroll
    for (int b = 0; b < NR; ++b) acc[a][b] = 0.0;
  const int* zl = g.zl;
  for (int bb = 0; bb < nb; ++bb) {
    const int s = pl * nb + bb;
    plane_zero<N>(P, NT);
    __syncthreads();
    plane_scatter<N>(P, pen + ((size_t)s * N + ix) * g.ncol_pad, g, NT);
    __syncthreads();
    fft_lines<N, +1, NT, N>(P, g.nza, LD, [zl](int f) { return zl[f]; }, NoPost{}, g.tw64);
    const Z64* ps = psi_r + ((size_t)(band0 + bb) * N + ix) * N * N;
    fft_lines<N, +1, NT, N>(
        P, N, 1, [](int f) { return f * LD; },
        [&acc, ps](int f, int n, int slot, int r, Z64 v) {
          const Z64 w = ps[f * N + n];
          acc[slot][r] += w.re * v.re + w.im * v.im;
          return v;
        },
        g.tw64);
  }
  double* dp = dn + ((size_t)pert_out[pl] * N + ix) * N * N;
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NSLOT; ++k) {
    if constexpr (R2 == 1) {
      const int f = tid + k * NT;
      if (f < N) {
#pragma unroll
        for (int r = 0; r < R1; ++r) dp[f * N + r] = scale * acc[k][r];
      }
    } else {
      const int it = tid + k * NT;
      if (it < N * R1) {
        const int f = it / R1, j = it - f * R1;
#pragma unroll
        for (int r = 0; r < R2; ++r) dp[f * N + j + r * R1] = scale * acc[k][r];
      }
    }
  }
}

// Raise the dynamic LDS limit of a plane kernel once per instantiation.
void set_lds(const void* kernel, size_t bytes) {
  static const void* done[64];
  static int ndone = 0;
  if (bytes <= 64 * 1024) return;
  for (int i = 0; i < ndone; ++i)
    if (done[i] == kernel) return;
  (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (ndone < 64) done[ndone++] = kernel;
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

size_t plane_lds_bytes(int N, int elem_bytes) { return (size_t)N * (N + 1) * elem_bytes; }

#define STERN_DISPATCH_N(N_, CALL)                  \
  switch (N_) {                                     \
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
    default: break;                                 \
  }

void launch_xinv(const FftGeom& g, const Z64* sph, const int* vidx, int nvec, Z64* pen, hipStream_t st) {
  if (nvec <= 0) return;
  dim3 grid(g.ncol_pad / kColBlock, nvec);
  STERN_DISPATCH_N(g.N, (k_xinv<NN><<<grid, kXThreads, 0, st>>>(sph, vidx, pen, g)));
}

void launch_xfwd(const FftGeom& g, const Z64* pen, const int* vidx, int nvec, Z64* out, int mode, const Z64* pin,
                 const double* eps, double scale, hipStream_t st) {
  if (nvec <= 0) return;
  dim3 grid(g.ncol_pad / kColBlock, nvec);
  if (mode == 0) {
    STERN_DISPATCH_N(g.N, (k_xfwd<NN, 0><<<grid, kXThreads, 0, st>>>(pen, vidx, out, pin, eps, scale, g)));
  } else if (mode == 1) {
    STERN_DISPATCH_N(g.N, (k_xfwd<NN, 1><<<grid, kXThreads, 0, st>>>(pen, vidx, out, pin, eps, scale, g)));
  } else {
    STERN_DISPATCH_N(g.N, (k_xfwd<NN, 2><<<grid, kXThreads, 0, st>>>(pen, vidx, out, pin, eps, scale, g)));
  }
}

void launch_plane_vloc(const FftGeom& g, Z64* pen, const int* vidx, int nvec, const double* v_r, hipStream_t st) {
  if (nvec <= 0) return;
  const size_t lds = plane_lds_bytes(g.N, sizeof(Z64));
  dim3 grid(g.N, nvec);
  STERN_DISPATCH_N(g.N, (set_lds((const void*)k_plane_vloc<NN>, lds),
                         k_plane_vloc<NN><<<grid, plane_threads<NN>(), lds, st>>>(pen, vidx, v_r, g)));
}

void launch_plane_rhs(const FftGeom& g, const Z64* psi_r, const double* dv, const int* band, const int* pert,
                      int nvec, Z64* pen, hipStream_t st) {
  if (nvec <= 0) return;
  const size_t lds = plane_lds_bytes(g.N, sizeof(Z64));
  dim3 grid(g.N, nvec);
  STERN_DISPATCH_N(g.N, (set_lds((const void*)k_plane_rhs<NN>, lds),
                         k_plane_rhs<NN><<<grid, plane_threads<NN>(), lds, st>>>(psi_r, dv, band, pert, pen, g)));
}

void launch_plane_full_inv(const FftGeom& g, const Z64* pen, int nvec, Z64* out, hipStream_t st) {
  if (nvec <= 0) return;
  const size_t lds = plane_lds_bytes(g.N, sizeof(Z64));
  dim3 grid(g.N, nvec);
  STERN_DISPATCH_N(g.N, (set_lds((const void*)k_plane_full_inv<NN>, lds),
                         k_plane_full_inv<NN><<<grid, plane_threads<NN>(), lds, st>>>(pen, out, g)));
}

void launch_plane_dn(const FftGeom& g, const Z64* pen, const Z64* psi_r, int band0, int nb, int npert,
                     const int* pert_out, double scale, double* dn, hipStream_t st) {
  if (npert <= 0 || nb <= 0) return;
  const size_t lds = plane_lds_bytes(g.N, sizeof(Z64));
  dim3 grid(g.N, npert);
  STERN_DISPATCH_N(g.N, (set_lds((const void*)k_plane_dn<NN>, lds),
                         k_plane_dn<NN><<<grid, plane_threads<NN>(), lds, st>>>(pen, psi_r, band0, nb, pert_out,
                                                                               scale, dn, g)));
}

}  // namespace stern
