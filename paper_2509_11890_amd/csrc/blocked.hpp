// Blocked (GEMM-based) dense Cholesky, triangular solves and LU for the local
// direct solves of large frames.
#pragma once

#include "tt.hpp"

namespace ttipm {

struct BlockedFactors {
  int n = 0;
  int nb = 32;
  DevBuf dinv;   // inverses of the lower diagonal blocks (Cholesky: L_jj, LU: unit L_jj)
  DevBuf uinv;   // LU: inverses of the upper diagonal blocks
  DevBuf piv;    // LU: row pivots (ints)
};

// In-place Cholesky (lower, row-major n x n).  Returns 0 or j+1 for a non-positive pivot.
int chol_blocked(double* A, int n, BlockedFactors& f, Ctx& c);
// Solve L X = B (trans = false) or L^T X = B (trans = true) in place, B row-major n x nrhs.
void trsm_blocked(const double* L, int n, const BlockedFactors& f, double* B, int nrhs, bool trans, Ctx& c);
// In-place LU with partial pivoting (row-major n x n).  Returns 0 or j+1 for a zero pivot.
int lu_blocked(double* A, int n, BlockedFactors& f, Ctx& c);
// Solve A X = B with the factors of lu_blocked (B row-major n x nrhs, in place).
void lu_solve_blocked(const double* A, int n, const BlockedFactors& f, double* B, int nrhs, Ctx& c);

}  // namespace ttipm
