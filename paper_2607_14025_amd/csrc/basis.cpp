// Host-side basis construction (sphere, pencil columns, V_loc on the grid, KB rows).
#include "basis.hpp"

#include <algorithm>
#include <cmath>
#include <tuple>

namespace stern {

namespace {
constexpr double kTwoPi = 6.283185307179586476925286766559;

bool smooth23(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}
int imod(int a, int n) { return ((a % n) + n) % n; }
// largest m >= 0 with m^2 <= v (v >= 0)
int isqrt_floor(double v) {
  int m = (int)std::floor(std::sqrt(v));
  while ((double)(m + 1) * (m + 1) <= v) ++m;
  while (m > 0 && (double)m * m > v) --m;
  return m;
}
}  // namespace

int default_fft_n(double L, double ecut) {
  const int nmax = (int)std::floor(2.0 * std::sqrt(ecut) * L / kTwoPi);
  int n = 2 * (nmax + 1) + 1;
  while (!smooth23(n)) ++n;
  return n;
}

std::string build_basis(const CellParams& c, HostBasis& hb, bool sphere_only) {
  if (!(c.L > 0) || !(c.ecut > 0)) return "L and ecut must be positive";
  hb = HostBasis();
  hb.L = c.L;
  hb.ecut = c.ecut;
  hb.omega = c.L * c.L * c.L;
  hb.b = kTwoPi / c.L;
  hb.N = c.fft_n > 0 ? c.fft_n : default_fft_n(c.L, c.ecut);
  const double r2 = c.ecut * c.L * c.L / (kTwoPi * kTwoPi);
  const int nm = isqrt_floor(r2);
  const int N = hb.N;
  // The grid holds the 4 Ecut sphere of V_loc (|n| <= nq = floor(2 sqrt(r2))) without
  // aliasing, so V_loc(r) is exact in the basis. As nq >= 2 nm this also gives
  // N >= 4 nm + 1, which the compact plane kernels take as given: they skip the y and z
  // ranges outside [0, (N - 1) / 4] and [N - (N - 1) / 4, N) without a test.
  const int nq = isqrt_floor(4.0 * r2);
  if (N < (sphere_only ? 2 * nm + 1 : 2 * nq + 1)) return "fft_n too small for the 4 ecut sphere";

  // canonical order: |n|^2, then n_x, n_y, n_z
  std::vector<std::tuple<int, int, int, int>> pts;
  for (int a = -nm; a <= nm; ++a)
    for (int b = -nm; b <= nm; ++b)
      for (int d = -nm; d <= nm; ++d) {
        const int n2 = a * a + b * b + d * d;
        if ((double)n2 <= r2) pts.emplace_back(n2, a, b, d);
      }
  std::sort(pts.begin(), pts.end());
  hb.npw = (int)pts.size();
  hb.npw_pad = (hb.npw + 63) / 64 * 64;
  hb.miller.resize(3 * (size_t)hb.npw);
  for (int k = 0; k < hb.npw; ++k) {
    hb.miller[3 * k] = std::get<1>(pts[k]);
    hb.miller[3 * k + 1] = std::get<2>(pts[k]);
    hb.miller[3 * k + 2] = std::get<3>(pts[k]);
  }

  // x-pencil columns (n_y, n_z), ordered by n_y then n_z; n_x contiguous inside
  std::vector<int> colid((2 * nm + 1) * (2 * nm + 1), -1);
  int start = 0;
  for (int ny = -nm; ny <= nm; ++ny)
    for (int nz = -nm; nz <= nm; ++nz) {
      const double rest = r2 - (double)(ny * ny + nz * nz);
      if (rest < 0) continue;
      const int xm = isqrt_floor(rest);
      colid[(ny + nm) * (2 * nm + 1) + (nz + nm)] = hb.ncol;
      hb.col_start.push_back(start);
      hb.col_len.push_back(2 * xm + 1);
      hb.col_xmin.push_back(-xm);
      hb.col_pos.push_back(imod(ny, N) * N + imod(nz, N));
      start += 2 * xm + 1;
      ++hb.ncol;
    }
  if (start != hb.npw) return "internal error: column count mismatch";
  hb.ncol_pad = (hb.ncol + kColPad - 1) / kColPad * kColPad;
  hb.col_start.resize(hb.ncol_pad, 0);
  hb.col_len.resize(hb.ncol_pad, 0);
  hb.col_xmin.resize(hb.ncol_pad, 0);
  for (int nz = -nm; nz <= nm; ++nz) hb.zl.push_back(imod(nz, N));
  std::sort(hb.zl.begin(), hb.zl.end());
  hb.nza = (int)hb.zl.size();
  hb.zact_lo = nm;
  hb.zact_hi = N - nm;
  hb.ycol.assign((size_t)hb.nza * N, -1);
  for (int f = 0; f < hb.nza; ++f) {
    const int iz = hb.zl[f];
    const int nz = (2 * iz < N) ? iz : iz - N;
    for (int iy = 0; iy < N; ++iy) {
      const int ny = (2 * iy < N) ? iy : iy - N;
      if (ny < -nm || ny > nm) continue;
      hb.ycol[(size_t)iy * hb.nza + f] = colid[(ny + nm) * (2 * nm + 1) + (nz + nm)];
    }
  }

  hb.perm.resize(hb.npw);
  hb.g2h.assign(hb.npw_pad, 0.0);
  for (int k = 0; k < hb.npw; ++k) {
    const int nx = hb.miller[3 * k], ny = hb.miller[3 * k + 1], nz = hb.miller[3 * k + 2];
    const int cid = colid[(ny + nm) * (2 * nm + 1) + (nz + nm)];
    const int idx = hb.col_start[cid] + (nx - hb.col_xmin[cid]);
    hb.perm[k] = idx;
    hb.g2h[idx] = 0.5 * hb.b * hb.b * (double)(nx * nx + ny * ny + nz * nz);
  }
  return std::string();
}

std::vector<double> vloc_grid(const CellParams& c, const HostBasis& hb, double scale) {
  using cd = std::complex<double>;
  const int N = hb.N;
  const double r2 = c.ecut * c.L * c.L / (kTwoPi * kTwoPi);
  const int nq = isqrt_floor(4.0 * r2);
  const int W = 2 * nq + 1;
  const int na = (int)(c.pos.size() / 3);
  const double b = hb.b;
  const double pref = c.amp * std::pow(kTwoPi * c.sigma * c.sigma, 1.5) / hb.omega;
  // 1-D structure-factor phases exp(-i b n R_a) per axis
  std::vector<cd> ph(3 * (size_t)na * W);
  for (int a = 0; a < na; ++a)
    for (int ax = 0; ax < 3; ++ax)
      for (int n = -nq; n <= nq; ++n) {
        const double t = -b * n * c.pos[3 * a + ax];
        ph[((size_t)ax * na + a) * W + (n + nq)] = cd(std::cos(t), std::sin(t));
      }
  std::vector<cd> vq((size_t)W * W * W, cd(0, 0));
  for (int nx = -nq; nx <= nq; ++nx)
    for (int ny = -nq; ny <= nq; ++ny)
      for (int nz = -nq; nz <= nq; ++nz) {
        const int n2 = nx * nx + ny * ny + nz * nz;
        if ((double)n2 > 4.0 * r2) continue;
        cd s(0, 0);
        for (int a = 0; a < na; ++a)
          s += ph[((size_t)0 * na + a) * W + nx + nq] * ph[((size_t)1 * na + a) * W + ny + nq] *
               ph[((size_t)2 * na + a) * W + nz + nq];
        const double g2 = b * b * n2;
        vq[((size_t)(nx + nq) * W + (ny + nq)) * W + (nz + nq)] =
            pref * std::exp(-0.5 * c.sigma * c.sigma * g2) * s;
      }
  std::vector<cd> tw(N);
  for (int m = 0; m < N; ++m) tw[m] = cd(std::cos(kTwoPi * m / N), std::sin(kTwoPi * m / N));
  // z: F1[nx][ny][jz]
  std::vector<cd> f1((size_t)W * W * N, cd(0, 0));
  for (int ix = 0; ix < W; ++ix)
    for (int iy = 0; iy < W; ++iy) {
      const cd* src = &vq[((size_t)ix * W + iy) * W];
      cd* dst = &f1[((size_t)ix * W + iy) * N];
      for (int iz = 0; iz < W; ++iz) {
        if (src[iz] == cd(0, 0)) continue;
        const int nz = imod(iz - nq, N);
        for (int jz = 0; jz < N; ++jz) dst[jz] += src[iz] * tw[(size_t)nz * jz % N];
      }
    }
  // y: F2[nx][jy][jz]
  std::vector<cd> f2((size_t)W * N * N, cd(0, 0));
  for (int ix = 0; ix < W; ++ix)
    for (int iy = 0; iy < W; ++iy) {
      const int ny = imod(iy - nq, N);
      const cd* src = &f1[((size_t)ix * W + iy) * N];
      for (int jy = 0; jy < N; ++jy) {
        const cd w = tw[(size_t)ny * jy % N];
        cd* dst = &f2[((size_t)ix * N + jy) * N];
        for (int jz = 0; jz < N; ++jz) dst[jz] += src[jz] * w;
      }
    }
  // x: V[jx][jy][jz]
  std::vector<cd> v((size_t)N * N * N, cd(0, 0));
  for (int ix = 0; ix < W; ++ix) {
    const int nx = imod(ix - nq, N);
    const cd* src = &f2[(size_t)ix * N * N];
    for (int jx = 0; jx < N; ++jx) {
      const cd w = tw[(size_t)nx * jx % N];
      cd* dst = &v[(size_t)jx * N * N];
      for (size_t t = 0; t < (size_t)N * N; ++t) dst[t] += src[t] * w;
    }
  }
  std::vector<double> out((size_t)N * N * N);
  for (size_t t = 0; t < out.size(); ++t) out[t] = scale * v[t].real();
  return out;
}

std::vector<std::complex<double>> kb_projectors(const CellParams& c, const HostBasis& hb, int n_rows) {
  using cd = std::complex<double>;
  const int na = (int)(c.pos.size() / 3);
  std::vector<cd> B((size_t)n_rows * hb.npw_pad, cd(0, 0));
  const double inv = 1.0 / std::sqrt(hb.omega);
  for (int k = 0; k < hb.npw; ++k) {
    const int idx = hb.perm[k];
    const double gx = hb.b * hb.miller[3 * k], gy = hb.b * hb.miller[3 * k + 1], gz = hb.b * hb.miller[3 * k + 2];
    const double rad = inv * std::exp(-0.5 * c.width * c.width * (gx * gx + gy * gy + gz * gz));
    for (int a = 0; a < na; ++a) {
      const double t = -(gx * c.pos[3 * a] + gy * c.pos[3 * a + 1] + gz * c.pos[3 * a + 2]);
      B[(size_t)a * hb.npw_pad + idx] = rad * cd(std::cos(t), std::sin(t));
    }
  }
  return B;
}

}  // namespace stern
