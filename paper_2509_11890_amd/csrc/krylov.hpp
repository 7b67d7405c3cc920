// Restarted GMRES for the local systems (Sec. 3.3), with optional right
// preconditioning and a mixed-precision mode in which the Arnoldi products use
// BF16-operand contractions while every restart recomputes the true residual
// in FP64 (GMRES as the inner solver of an iterative refinement).
#pragma once

#include <functional>

#include "tt.hpp"

namespace ttipm {

struct KrylovOps {
  // y = K x; low = true asks for the low-precision (BF16-operand) product
  std::function<void(const double* x, double* y, bool low)> matvec;
  // y = M^{-1} x (right preconditioner); empty = identity
  std::function<void(const double* x, double* y)> precond;
};

struct KrylovParams {
  double rtol = 1e-10;    // target ||f - K u|| <= rtol ||f|| (FP64 residual)
  int restart = 40;
  int maxit = 400;        // total Arnoldi steps
  bool mixed = false;     // low-precision Arnoldi products + FP64 refinement at restarts
  double inner_tol = 1e-2;  // mixed: per-cycle residual reduction asked from the inner solve
};

struct KrylovInfo {
  int iters = 0;
  int cycles = 0;
  double rel_res = 0.0;   // final FP64 relative residual
};

// Solve K u = f; u holds the initial guess on entry.
void gmres_solve(long n, const KrylovOps& ops, const double* f, double* u, const KrylovParams& prm, KrylovInfo& info,
                 Ctx& c);

// Block-Jacobi preconditioner of an L-component local operator on [L][r][m][s]
// vectors: one (L m) x (L m) block per rank pair (a, b), holding the diagonal
// entries phiL[a][.][a] and phiR[b][.][b] of every projected operator.
struct BlockJacobi {
  int r = 0, s = 0, m = 0, L = 0;
  DevBuf blk;   // [(a, b)][L m][L m]: assembled blocks, then their inverses
  void init(int r_, int s_, int m_, int L_, Ctx& c);
  void copy_from(const BlockJacobi& o, Ctx& c);
  // blocks[row][col] += coeff * D, D the diagonal block of the chain (applied first to last)
  struct Op {
    const double* phiL;   // [r][R][r]
    const double* core;   // [R][m][m][Rp] (row-major), nullptr = identity (R = Rp = 1)
    const double* phiR;   // [s][Rp][s]
    int R, Rp;
  };
  void add(int row, int col, double coeff, const Op* chain, int nchain, Ctx& c);
  void invert(Ctx& c);                                        // in place; singular blocks become identity
  void apply(const double* x, double* y, Ctx& c) const;       // y = M^{-1} x
};

}  // namespace ttipm
