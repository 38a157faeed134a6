// Cyclic Jacobi eigensolvers (Golub and Van Loan, Matrix Computations, ch. 8) for the projected
// matrices of the PDEP and Liouville Davidson iterations.
#include "hostla.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace stern {

// Eigenvalues (ascending) and eigenvectors (columns of V, row-major n x n) of a
// real symmetric matrix by cyclic Jacobi rotations.
void jacobi_eigh(std::vector<double> A, int n, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        // rotation angle that zeroes a(p, q): tan(2 t) = 2 apq / (aqq - app)
        const double theta = 0.5 * (a(q, q) - a(p, p)) / apq;
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - sn * akq;
          a(k, q) = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - sn * aqk;
          a(q, k) = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + c * vkq;
        }
      }
  }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int i, int j) { return a(i, i) < a(j, j); });
  w.resize(n);
  std::vector<double> Vs((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    w[c] = a(ord[c], ord[c]);
    for (int k = 0; k < n; ++k) Vs[(size_t)k * n + c] = V[(size_t)k * n + ord[c]];
  }
  V.swap(Vs);
}

// Eigenpairs of a small Hermitian matrix by cyclic Jacobi rotations (host): A [n][n] row-major,
// w ascending, V [n][n] with the eigenvectors as columns. Each rotation first takes the phase of
// a_pq into the q column, then zeroes the now real off-diagonal pair as in the real case.
void jacobi_zheev(std::vector<std::complex<double>> A, int n, std::vector<double>& w,
                         std::vector<std::complex<double>>& V) {
  using cd = std::complex<double>;
  V.assign((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += std::norm(a(i, j));
        if (i != j) off += std::norm(a(i, j));
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double r = std::abs(a(p, q));
        if (r < 1e-300) continue;
        const cd ph = a(p, q) / r;  // e^{i phi}
        const double th = 0.5 * (a(q, q).real() - a(p, p).real()) / r;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // U = diag(1, e^{-i phi}) [[c, s], [-s, c]]: A <- U^H A U, V <- V U
        const cd upp = c, upq = s, uqp = -s * std::conj(ph), uqq = c * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // columns
          const cd x = a(k, p), y = a(k, q);
          a(k, p) = x * upp + y * uqp;
          a(k, q) = x * upq + y * uqq;
        }
        for (int k = 0; k < n; ++k) {  // rows
          const cd x = a(p, k), y = a(q, k);
          a(p, k) = std::conj(upp) * x + std::conj(uqp) * y;
          a(q, k) = std::conj(upq) * x + std::conj(uqq) * y;
        }
        a(p, q) = a(q, p) = 0.0;
        a(p, p) = a(p, p).real();
        a(q, q) = a(q, q).real();
        for (int k = 0; k < n; ++k) {
          const cd x = V[(size_t)k * n + p], y = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = x * upp + y * uqp;
          V[(size_t)k * n + q] = x * upq + y * uqq;
        }
      }
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
  std::vector<std::complex<double>> Vs((size_t)n * n);
  w.resize(n);
  for (int j = 0; j < n; ++j) {
    w[j] = a(ord[j], ord[j]).real();
    for (int k = 0; k < n; ++k) Vs[(size_t)k * n + j] = V[(size_t)k * n + ord[j]];
  }
  V.swap(Vs);
}

}  // namespace stern
