// Small dense complex eigenproblems on the host (subspace matrices of the
// Davidson iteration).
#pragma once
#include <complex>
#include <vector>

namespace lrcc {

// Eigenvalues w[n] and right eigenvectors V[n*n] (column k = vector of w[k], unit
// 2-norm) of a general complex matrix A[n*n] (row-major).  Householder reduction
// to Hessenberg form, shifted QR iteration to the Schur form, back substitution.
// Returns false if the QR iteration does not converge.
bool small_eig(int n, std::vector<std::complex<double>> A, std::vector<std::complex<double>> &w,
               std::vector<std::complex<double>> &V);

}  // namespace lrcc
