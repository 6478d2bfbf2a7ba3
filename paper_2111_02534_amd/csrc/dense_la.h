// Small dense host linear algebra (row-major double arrays).
#pragma once

namespace tp3b {

// Upper Hessenberg form H = Z^T A Z in place; Z row-major n x n or null.
void hessenberg(int n, double* A, double* Z);
// Real Schur form of A (overwritten by the quasi-triangular T); Z receives the
// orthogonal Schur vectors (A_in = Z T Z^T) when not null.
bool real_schur(int n, double* A, double* Z, double* wr, double* wi);
// Ordered real Schur form of M (m x m): M S = S T, eigenvalues ascending by real
// part; pair_start[i] = 1 where a 2x2 block (complex pair) starts.
bool ordered_schur(int m, const double* M, double* S, double* T, int* pair_start);
// A = S diag(lam) S^{-1} for a matrix with real spectrum; false otherwise.
bool eigen_decompose_real(int n, const double* A, double* S, double* Sinv, double* lam);
bool lu_inverse(int n, const double* A, double* Ainv);
// Least squares min ||beta e1 - H y|| for the (k+1) x k Hessenberg H.
void hessenberg_lstsq(int k, const double* H, int ldh, double beta, double* y);

}  // namespace tp3b
