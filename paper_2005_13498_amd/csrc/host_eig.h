// Small dense symmetric eigenproblems on the host (Lanczos Ritz values).
#pragma once

#include <vector>

namespace hub {

// Eigenvalues (ascending) and orthonormal eigenvectors of the real symmetric
// n x n matrix A (row-major), by cyclic Jacobi rotations: each rotation
// zeroes one off-diagonal pair; sweeps repeat until the off-diagonal mass
// is below 1e-30 of the total.  vecs[i*n + k] = component i of vector k.
void sym_eig(int n, std::vector<double> A, std::vector<double>& vals, std::vector<double>& vecs);

}  // namespace hub
