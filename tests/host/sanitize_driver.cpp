// The library's host code built under AddressSanitizer and UndefinedBehaviorSanitizer (by
// tests/test_host_sanitizers.py with g++): the plane-wave basis, the local potential on the grid
// and the projector rows of the cells read from stdin ("L ecut n_atoms fft_n" per line, fft_n 0 for
// the default grid), with consistency checks, then the dense Jacobi eigensolvers on seeded random
// matrices. Prints one line per cell and per matrix; exits non-zero on a failed check.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "basis.hpp"
#include "hostla.hpp"

using namespace stern;

static int check_cell(double L, double ecut, int na, int fft_n, std::mt19937_64& rng) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  CellParams c;
  c.L = L;
  c.ecut = ecut;
  c.fft_n = fft_n;
  for (int i = 0; i < 3 * na; ++i) c.pos.push_back(L * u(rng));
  HostBasis hb;
  const std::string e = build_basis(c, hb);
  if (!e.empty()) {
    printf("cell L %g ecut %g: %s\n", L, ecut, e.c_str());
    return 0;
  }
  // perm is a permutation of the column-order slots below npw; columns tile [0, npw)
  std::vector<char> seen(hb.npw_pad, 0);
  for (int k = 0; k < hb.npw; ++k) {
    const int p = hb.perm[k];
    if (p < 0 || p >= hb.npw || seen[p]) return 10;
    seen[p] = 1;
  }
  long covered = 0;
  for (int col = 0; col < hb.ncol_pad; ++col) covered += hb.col_len[col];
  if (covered != hb.npw) return 11;
  for (int k = hb.npw; k < hb.npw_pad; ++k)
    if (hb.g2h[k] != 0.0) return 12;
  const std::vector<double> v = vloc_grid(c, hb, 1.0);
  if (v.size() != (size_t)hb.N * hb.N * hb.N) return 13;
  for (double x : v)
    if (!std::isfinite(x)) return 14;
  const int rows = (na + 63) / 64 * 64;
  const std::vector<std::complex<double>> B = kb_projectors(c, hb, rows);
  if (B.size() != (size_t)rows * hb.npw_pad) return 15;
  for (int r = na; r < rows; ++r)
    for (int k = 0; k < hb.npw_pad; ++k)
      if (B[(size_t)r * hb.npw_pad + k] != std::complex<double>(0.0, 0.0)) return 16;
  printf("cell L %g ecut %g atoms %d: N %d npw %d npw_pad %d ncol %d nza %d\n", L, ecut, na, hb.N, hb.npw,
         hb.npw_pad, hb.ncol, hb.nza);
  return 0;
}

static int check_jacobi(int n, std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  std::vector<double> A((size_t)n * n);
  std::vector<std::complex<double>> H((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      A[(size_t)i * n + j] = A[(size_t)j * n + i] = nd(rng);
      const std::complex<double> z(nd(rng), i == j ? 0.0 : nd(rng));
      H[(size_t)i * n + j] = z;
      H[(size_t)j * n + i] = std::conj(z);
    }
  std::vector<double> w, V;
  jacobi_eigh(A, n, w, V);
  std::vector<double> wz;
  std::vector<std::complex<double>> Vz;
  jacobi_zheev(H, n, wz, Vz);
  double ra = 0.0, rz = 0.0, oa = 0.0, oz = 0.0;
  for (int k = 0; k < n; ++k) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      std::complex<double> t = 0.0;
      for (int j = 0; j < n; ++j) {
        s += A[(size_t)i * n + j] * V[(size_t)j * n + k];
        t += H[(size_t)i * n + j] * Vz[(size_t)j * n + k];
      }
      ra = std::max(ra, std::fabs(s - w[k] * V[(size_t)i * n + k]));
      rz = std::max(rz, std::abs(t - wz[k] * Vz[(size_t)i * n + k]));
    }
    for (int l = 0; l < n; ++l) {
      double s = 0.0;
      std::complex<double> t = 0.0;
      for (int j = 0; j < n; ++j) {
        s += V[(size_t)j * n + k] * V[(size_t)j * n + l];
        t += std::conj(Vz[(size_t)j * n + k]) * Vz[(size_t)j * n + l];
      }
      oa = std::max(oa, std::fabs(s - (k == l ? 1.0 : 0.0)));
      oz = std::max(oz, std::abs(t - (k == l ? 1.0 : 0.0)));
    }
  }
  for (int k = 1; k < n; ++k)
    if (w[k] < w[k - 1] || wz[k] < wz[k - 1]) return 20;
  printf("jacobi n %d: real residual %.1e orthogonality %.1e; hermitian residual %.1e orthogonality %.1e\n", n, ra, oa,
         rz, oz);
  return (ra > 1e-10 * n || rz > 1e-10 * n || oa > 1e-12 * n || oz > 1e-12 * n) ? 21 : 0;
}

int main() {
  std::mt19937_64 rng(11);
  double L, ecut;
  int na, fft_n;
  while (scanf("%lf %lf %d %d", &L, &ecut, &na, &fft_n) == 4) {
    const int rc = check_cell(L, ecut, na, fft_n, rng);
    if (rc) {
      printf("cell L %g ecut %g: check %d failed\n", L, ecut, rc);
      return rc;
    }
  }
  for (int n : {1, 2, 3, 7, 24, 48}) {
    const int rc = check_jacobi(n, rng);
    if (rc) return rc;
  }
  return 0;
}
