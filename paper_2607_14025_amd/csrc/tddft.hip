// Grid kernels of the TDDFT Liouville apply (Tamm-Dancoff; Sec. II.C.1, eq. bse_tddft): the
// band-summed transition densities rho_e = sum_v conj(psi_v) a_{e,v}, the Coulomb factor on the
// 4 Ecut sphere, the products V_e psi_v, and for the bare-exchange direct term the occupied pair
// densities conj(psi_w) psi_v whose potentials are the integrals tau_{wv} of eq. tau_u and the
// sums sum_w tau_{wv} a_{e,w}. All of it is streaming work on
// full N^3 grids (one read and one write per point and band), so the kernels are plain
// grid-stride loops with coalesced complex FP64 accesses; the FFTs between them are the
// library's pencil and plane kernels.
#include "kernels.hpp"

namespace stern {

namespace {

constexpr int kGridThreads = 256;

// rho[e][j] = scale sum_v conj(psi_r[v][j]) a_r[e nb + v][j], bands summed in order
__global__ __launch_bounds__(kGridThreads) void k_band_density(const Z64* __restrict__ psi_r,
                                                               const Z64* __restrict__ a_r, int nb, size_t n3,
                                                               double scale, Z64* __restrict__ rho) {
  const int e = blockIdx.y;
  const Z64* ae = a_r + (size_t)e * nb * n3;
  for (size_t j = (size_t)blockIdx.x * kGridThreads + threadIdx.x; j < n3; j += (size_t)gridDim.x * kGridThreads) {
    double re = 0.0, im = 0.0;
    for (int v = 0; v < nb; ++v) {
      const Z64 p = psi_r[(size_t)v * n3 + j], a = ae[(size_t)v * n3 + j];
      re += p.re * a.re + p.im * a.im;
      im += p.re * a.im - p.im * a.re;
    }
    rho[(size_t)e * n3 + j] = zmk(scale * re, scale * im);
  }
}

// c[i] *= fac / g2h[i mod K]; zero where g2h = 0 (G = 0 and the padding, whatever they held)
__global__ __launch_bounds__(kGridThreads) void k_coulomb(Z64* __restrict__ c, const double* __restrict__ g2h, int K,
                                                          size_t total, double fac) {
  for (size_t i = (size_t)blockIdx.x * kGridThreads + threadIdx.x; i < total; i += (size_t)gridDim.x * kGridThreads) {
    const double h = g2h[i % K];
    const Z64 v = c[i];
    c[i] = h > 0.0 ? zmk(fac / h * v.re, fac / h * v.im) : zmk(0.0, 0.0);
  }
}

// out[e nb + v][j] = v_r[e][j] psi_r[v][j] (- alpha acc[e nb + v][j] when acc is given)
__global__ __launch_bounds__(kGridThreads) void k_grid_mul(const Z64* __restrict__ v_r, const Z64* __restrict__ psi_r,
                                                           int nb, size_t n3, const Z64* __restrict__ acc,
                                                           double alpha, Z64* __restrict__ out) {
  const int row = blockIdx.y, e = row / nb, v = row - e * nb;
  const Z64* ve = v_r + (size_t)e * n3;
  const Z64* pv = psi_r + (size_t)v * n3;
  const Z64* ac = acc ? acc + (size_t)row * n3 : nullptr;
  Z64* o = out + (size_t)row * n3;
  for (size_t j = (size_t)blockIdx.x * kGridThreads + threadIdx.x; j < n3; j += (size_t)gridDim.x * kGridThreads) {
    const Z64 a = ve[j], p = pv[j];
    Z64 r = zmk(a.re * p.re - a.im * p.im, a.re * p.im + a.im * p.re);
    if (ac) {
      const Z64 c = ac[j];
      r = zmk(r.re - alpha * c.re, r.im - alpha * c.im);
    }
    o[j] = r;
  }
}

// pair densities of one occupied orbital with all of them: out[w][j] = scale conj(psi_r[w][j]) psi_r[v][j]
__global__ __launch_bounds__(kGridThreads) void k_pair_density(const Z64* __restrict__ psi_r, int v, size_t n3,
                                                               double scale, Z64* __restrict__ out) {
  const int w = blockIdx.y;
  const Z64* pw = psi_r + (size_t)w * n3;
  const Z64* pv = psi_r + (size_t)v * n3;
  Z64* o = out + (size_t)w * n3;
  for (size_t j = (size_t)blockIdx.x * kGridThreads + threadIdx.x; j < n3; j += (size_t)gridDim.x * kGridThreads) {
    const Z64 a = pw[j], b = pv[j];
    o[j] = zmk(scale * (a.re * b.re + a.im * b.im), scale * (a.re * b.im - a.im * b.re));
  }
}

// acc[e nb + v][j] = sum_w tau[w][j] a_r[e nb + w][j], w in order (tau[w] = tau_{wv} of one band v)
__global__ __launch_bounds__(kGridThreads) void k_exch_acc(const Z64* __restrict__ tau, const Z64* __restrict__ a_r,
                                                           int nb, int v, size_t n3, Z64* __restrict__ acc) {
  const int e = blockIdx.y;
  const Z64* ae = a_r + (size_t)e * nb * n3;
  Z64* o = acc + ((size_t)e * nb + v) * n3;
  for (size_t j = (size_t)blockIdx.x * kGridThreads + threadIdx.x; j < n3; j += (size_t)gridDim.x * kGridThreads) {
    double re = 0.0, im = 0.0;
    for (int w = 0; w < nb; ++w) {
      const Z64 t = tau[(size_t)w * n3 + j], a = ae[(size_t)w * n3 + j];
      re += t.re * a.re - t.im * a.im;
      im += t.re * a.im + t.im * a.re;
    }
    o[j] = zmk(re, im);
  }
}

// y[i] += x[i]
__global__ __launch_bounds__(kGridThreads) void k_add(Z64* __restrict__ y, const Z64* __restrict__ x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kGridThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kGridThreads) {
    const Z64 a = y[i], b = x[i];
    y[i] = zmk(a.re + b.re, a.im + b.im);
  }
}

// proj[r][a] = N^-3 sum_j w[a][j] rho[r][j] (one workgroup per (a, r), fixed order)
__global__ __launch_bounds__(kGridThreads) void k_scr_proj(const Z64* __restrict__ rho, const double* __restrict__ w,
                                                           int n, size_t n3, Z64* __restrict__ proj) {
  __shared__ double sre[kGridThreads / 64], sim[kGridThreads / 64];
  const int a = blockIdx.x, r = blockIdx.y;
  const Z64* x = rho + (size_t)r * n3;
  const double* wa = w + (size_t)a * n3;
  double re = 0.0, im = 0.0;
  for (size_t j = threadIdx.x; j < n3; j += kGridThreads) {
    const double f = wa[j];
    const Z64 v = x[j];
    re += f * v.re;
    im += f * v.im;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o);
    im += __shfl_xor(im, o);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sre[wave] = re;
    sim[wave] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, ti = 0.0;
    for (int k = 0; k < kGridThreads / 64; ++k) {
      tr += sre[k];
      ti += sim[k];
    }
    proj[(size_t)r * n + a] = zmk(tr / (double)n3, ti / (double)n3);
  }
}

// tau[r][j] += sum_a w[a][j] c[a] proj[r][a]
__global__ __launch_bounds__(kGridThreads) void k_scr_add(Z64* __restrict__ tau, const double* __restrict__ w,
                                                          const Z64* __restrict__ proj, const double* __restrict__ c,
                                                          int n, size_t n3) {
  const int r = blockIdx.y;
  Z64* t = tau + (size_t)r * n3;
  const Z64* p = proj + (size_t)r * n;
  for (size_t j = (size_t)blockIdx.x * kGridThreads + threadIdx.x; j < n3; j += (size_t)gridDim.x * kGridThreads) {
    double re = 0.0, im = 0.0;
    for (int a = 0; a < n; ++a) {
      const double f = w[(size_t)a * n3 + j] * c[a];
      re += f * p[a].re;
      im += f * p[a].im;
    }
    const Z64 v = t[j];
    t[j] = zmk(v.re + re, v.im + im);
  }
}

unsigned grid_blocks(size_t n, int per_row_rows) {
  // enough workgroups to fill the chip several times over, fewer when a launch has many rows
  const size_t want = std::max<size_t>(1, 2048 / (size_t)std::max(1, per_row_rows));
  return (unsigned)std::max<size_t>(1, std::min<size_t>((n + kGridThreads - 1) / kGridThreads, want));
}

}  // namespace

void launch_band_density(const Z64* psi_r, const Z64* a_r, int n_exc, int nb, size_t n3, double scale, Z64* rho,
                         hipStream_t st) {
  if (n_exc <= 0 || nb <= 0) return;
  dim3 grid(grid_blocks(n3, n_exc), n_exc);
  k_band_density<<<grid, kGridThreads, 0, st>>>(psi_r, a_r, nb, n3, scale, rho);
}

void launch_coulomb(Z64* c, const double* g2h, int K, int nvec, double fac, hipStream_t st) {
  const size_t total = (size_t)K * nvec;
  if (total == 0) return;
  k_coulomb<<<grid_blocks(total, 1), kGridThreads, 0, st>>>(c, g2h, K, total, fac);
}

void launch_grid_mul(const Z64* v_r, const Z64* psi_r, int n_exc, int nb, size_t n3, const Z64* acc, double alpha,
                     Z64* out, hipStream_t st) {
  if (n_exc <= 0 || nb <= 0) return;
  dim3 grid(grid_blocks(n3, n_exc * nb), n_exc * nb);
  k_grid_mul<<<grid, kGridThreads, 0, st>>>(v_r, psi_r, nb, n3, acc, alpha, out);
}

void launch_pair_density(const Z64* psi_r, int v, int nb, size_t n3, double scale, Z64* out, hipStream_t st) {
  if (nb <= 0) return;
  dim3 grid(grid_blocks(n3, nb), nb);
  k_pair_density<<<grid, kGridThreads, 0, st>>>(psi_r, v, n3, scale, out);
}

void launch_exch_acc(const Z64* tau, const Z64* a_r, int n_exc, int nb, int v, size_t n3, Z64* acc, hipStream_t st) {
  if (n_exc <= 0 || nb <= 0) return;
  dim3 grid(grid_blocks(n3, n_exc), n_exc);
  k_exch_acc<<<grid, kGridThreads, 0, st>>>(tau, a_r, nb, v, n3, acc);
}

void launch_add(Z64* y, const Z64* x, size_t n, hipStream_t st) {
  if (n == 0) return;
  k_add<<<grid_blocks(n, 1), kGridThreads, 0, st>>>(y, x, n);
}

void launch_scr_proj(const Z64* rho, const double* w, int n, int nrows, size_t n3, Z64* proj, hipStream_t st) {
  if (n <= 0 || nrows <= 0) return;
  k_scr_proj<<<dim3(n, nrows), kGridThreads, 0, st>>>(rho, w, n, n3, proj);
}

void launch_scr_add(Z64* tau, const double* w, const Z64* proj, const double* c, int n, int nrows, size_t n3,
                    hipStream_t st) {
  if (n <= 0 || nrows <= 0) return;
  k_scr_add<<<dim3(grid_blocks(n3, nrows), nrows), kGridThreads, 0, st>>>(tau, w, proj, c, n, n3);
}

}  // namespace stern
