// Dense eigensolvers of the small projected matrices of the Davidson iterations (host code,
// no GPU types): cyclic Jacobi rotations for real symmetric and complex Hermitian matrices.
#pragma once
#include <complex>
#include <vector>

namespace stern {

// Eigenvalues (ascending) and eigenvectors (columns of V, row-major n x n) of a real symmetric
// matrix A [n][n] (row-major).
void jacobi_eigh(std::vector<double> A, int n, std::vector<double>& w, std::vector<double>& V);
// The same for a complex Hermitian matrix.
void jacobi_zheev(std::vector<std::complex<double>> A, int n, std::vector<double>& w,
                  std::vector<std::complex<double>>& V);

}  // namespace stern
