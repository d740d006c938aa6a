// eigen.hpp -- host generalised symmetric-definite eigen-solver (FD factors).
#pragma once

namespace igasg {

// K U = M U diag(lam), U^T M U = I for symmetric K, M (dense row-major n x n,
// half-bandwidth bw; M positive definite).  U is row-major [n][n] with
// column k the k-th eigenvector; lam ascending.  Returns false on failure.
bool gen_eig_banded(int n, int bw, const double* K, const double* M, double* U, double* lam);

}  // namespace igasg
