// Small dense Hermitian eigenproblems on the host (Rayleigh-Ritz matrices of the
// eigensolver, at most a few hundred rows).
#pragma once
#include <complex>
#include <vector>

namespace cstar {

using zd = std::complex<double>;

// A (n x n, row-major, Hermitian) = V diag(w) V^H; w ascending, V columns
// (row-major V[i*n + j] = component i of eigenvector j).  Cyclic Jacobi with
// complex rotations; A is not modified.
void herm_eig(int n, const std::vector<zd> &A, std::vector<double> &w, std::vector<zd> &V);

}  // namespace cstar
