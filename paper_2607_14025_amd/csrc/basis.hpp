// Host-side basis of one cell: sphere, x-pencil columns, local potential on the
// grid and KB projectors (no GPU needed).
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace stern {

// the x-pencil column count is padded to a multiple of this (whole column blocks of the
// x passes, 32 FP32 or 16 FP64 columns)
constexpr int kColPad = 32;

struct CellParams {
  double L = 0, ecut = 0;
  std::vector<double> pos;  // [n_atoms][3]
  double amp = -2, sigma = 1, D = 1, width = 1;
  int fft_n = 0;
};

struct HostBasis {
  double L = 0, ecut = 0, omega = 0, b = 0;
  int N = 0;
  int npw = 0, npw_pad = 0;
  int ncol = 0, ncol_pad = 0, nza = 0;
  std::vector<int32_t> miller;   // canonical order [npw][3]
  std::vector<int> perm;         // canonical index -> column-order index
  std::vector<int> col_start, col_len, col_xmin;  // [ncol_pad]
  std::vector<int> col_pos;      // [ncol]
  std::vector<int> zl;           // [nza]
  std::vector<int> ycol;         // [N][nza] column of (iy, zl[f]) or -1
  int zact_lo = 0, zact_hi = 0;  // active z lines: iz <= zact_lo or iz >= zact_hi
  std::vector<double> g2h;       // [npw_pad], column order
};

// Smallest 2^a 3^b >= 2 (floor(2 sqrt(ecut) L / 2 pi) + 1) + 1.
int default_fft_n(double L, double ecut);
// Fills everything but needs no GPU. Returns an empty string or an error message.
// sphere_only: the grid only has to hold the wave-function sphere (N >= 2 nmax + 1),
// not the products of two wave functions (N >= 4 nmax + 1).
std::string build_basis(const CellParams& c, HostBasis& hb, bool sphere_only = false);
// V(r) on the grid, [ix][iy][iz], from V(q) on |q|^2 <= 4 ecut, multiplied by `scale`.
std::vector<double> vloc_grid(const CellParams& c, const HostBasis& hb, double scale);
// beta_a(G) rows [n_rows][npw_pad] in column order (rows >= n_atoms are zero).
std::vector<std::complex<double>> kb_projectors(const CellParams& c, const HostBasis& hb, int n_rows);

}  // namespace stern
