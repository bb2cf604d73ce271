// Small dense FP64 linear algebra for plan construction (host only).
// Column-major storage throughout: A(i, j) = a[i + j * lda].
#pragma once

#include <cstdint>
#include <vector>

namespace sht {
namespace la {

// Householder QR with column pivoting of the m x n matrix A (overwritten).
// Stops after step k when the largest remaining column norm is <= tol (absolute)
// or k == kmax.  On return: rank = k, perm[0..n) the column order (the first
// `rank` are the pivots), A's upper triangle holds R (rank x n, in pivoted
// column order).  Ties in the pivot choice go to the lowest column index.
int pivoted_qr(int m, int n, double *a, int lda, double tol, int kmax, std::vector<int> &perm,
               std::vector<double> *tau = nullptr);

// Solve R11 T = R12 for T (k x (n-k)), R11 = R(0:k, 0:k) upper triangular.
void solve_upper(int k, int n, const double *r, int ldr, double *t /* k x (n-k), ld k */);

// Orthonormal basis Q (m x k) of the first k pivoted columns after
// pivoted_qr: forms Q from the Householder reflectors stored below the
// diagonal of A and tau.
void form_q(int m, int k, const double *a, int lda, const std::vector<double> &tau, double *q /* m x k */);

// One-sided Jacobi SVD of the m x n matrix A (m >= n): A = U diag(s) V^T.
// A is overwritten by U (m x n); v is n x n; singular values descending.
void jacobi_svd(int m, int n, double *a, int lda, double *s, double *v);

// Moore-Penrose pseudo-inverse of the m x n matrix A (via the SVD), relative
// cutoff rcond on the singular values: out is n x m.
void pinv(int m, int n, const double *a, int lda, double rcond, double *out);

// C (m x n) = alpha * op(A) * op(B) + beta * C, op = transpose if flag set.
void gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *a, int lda,
          const double *b, int ldb, double beta, double *c, int ldc);

}  // namespace la
}  // namespace sht
