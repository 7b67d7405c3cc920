// Single-workgroup dense FP64 factorisations on the device.
#pragma once

#include "common.hpp"

namespace ttipm {

// Householder QR of column-major A (m x n, lda): R upper, reflectors below, tau[min(m,n)].
void dense_qr(double* A, int m, int n, int lda, double* tau, hipStream_t s);
// Explicit first k columns of Q (column-major, ldq) from dense_qr output.
void dense_qr_form_q(const double* A, int m, int n, int lda, const double* tau, double* Q, int k, int ldq,
                     hipStream_t s);
// One-sided Jacobi SVD of column-major A (m x n, lda = m, destroyed):
// U (m x n col-major), sigma[n] descending, V (n x n col-major).  Column
// pairs count as orthogonal below max(tol, 4 eps sqrt(m)) relative.
// work >= n*n doubles, iwork >= n + 1 ints (iwork[n] = sweeps used).
void dense_svd(double* A, int m, int n, double* U, double* sigma, double* V, double* work, int* iwork,
               hipStream_t s, int max_sweeps = 40, double tol = 4e-16);
// True when dense_svd of an m x n matrix keeps both A and V in LDS.
bool dense_svd_fits_lds(int m, int n);
// The same sweeps without accumulating the rotations: U (m x n col-major) and
// sigma[n] descending only; A is destroyed unless it fits in LDS.  n <= 4096.
// iwork >= n + 1 ints (iwork[n] = sweeps used).
void dense_svd_left(double* A, int m, int n, double* U, double* sigma, int* iwork, hipStream_t s,
                    int max_sweeps = 40, double tol = 4e-16);
// True when dense_svd_left of an m x n matrix keeps A in LDS.
bool dense_svd_left_fits_lds(int m, int n);
// Smallest eigenpair of a symmetric row-major p x p matrix B (restarted Lanczos
// with full reorthogonalisation): v (p, unit norm), lam (1 double, device).
// With v_init, v holds the start vector on entry (a warm start; a zero vector
// falls back to the fixed pseudo-random start).
// work >= p * (min(kmax, p) + 1) doubles.
void dense_sym_min_eig(const double* B, int p, double* v, double* lam, double* work, hipStream_t s,
                       int kmax = 128, int restarts = 8, double tol = 1e-12, bool v_init = false);
// LU with partial pivoting; solves A X = B in place (row-major).  status[0] != 0 on a zero pivot.
void dense_lu_solve(double* A, int n, double* B, int nrhs, int* status, hipStream_t s);
// True when the LDS-resident Cholesky / LU-solve kernels take an n x n matrix
// (and n x nrhs right-hand sides); larger matrices go through the blocked
// factorisations instead.
bool dense_small_fits_lds(int n, int nrhs = 1);
// Cholesky (lower, row-major, in place).  status[0] = j+1 if not positive definite.
void dense_cholesky(double* A, int n, int* status, hipStream_t s);
// A <- (A + A^T) / 2 (row-major n x n).
void dense_symmetrize(double* A, int n, hipStream_t s);
// Solve L X = B (or L^T X = B) in place; L lower triangular row-major.
void dense_trsm_lower(const double* L, int n, double* B, int nrhs, bool transpose, hipStream_t s);
// Solve L^T L X = B in place (both sweeps in one launch where the slab fits LDS).
void dense_chol_solve(const double* L, int n, double* B, int nrhs, hipStream_t s);

}  // namespace ttipm
