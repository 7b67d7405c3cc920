// Strided batched GEMM on MFMA (FP64, or BF16 operands with FP32 accumulation).
#pragma once

#include "common.hpp"

namespace ttipm {

// C[b](m, n) = alpha * sum_k A[b](m, k) B[b](k, n) + beta * C[b](m, n)
// with element addresses A + b*sA + m*am + k*ak (same pattern for B and C).
struct Gemm {
  int M = 0, N = 0, K = 0, batch = 1;
  const double* A = nullptr; long am = 0, ak = 0, sA = 0;
  const double* B = nullptr; long bk = 0, bn = 0, sB = 0;
  double* C = nullptr; long cm = 0, cn = 0, sC = 0;
  double alpha = 1.0, beta = 0.0;
};

enum class GemmPrec { F64, BF16 };

// Scratch for split-K partial sums; grows on demand, or (fixed != nullptr) a
// caller-provided region of fixed_n doubles that is never grown.
struct Workspace {
  DevBuf buf;
  double* fixed = nullptr;
  size_t fixed_n = 0;
  double* take(size_t n);
};

// Upper bound (doubles) of the split-K partials one problem needs in gemm()
// or in a grouped launch; a gemm_grouped call needs at most the sum over its
// problems.
size_t gemm_splitk_need(const Gemm& q, GemmPrec prec);

void gemm(const Gemm& g, hipStream_t stream, Workspace* ws = nullptr, GemmPrec prec = GemmPrec::F64);

// Independent products in one launch (up to 8 with the same operand layouts;
// the others go through gemm()), FP64 or BF16 operands.  Outputs must not
// overlap: the problems run concurrently.
void gemm_grouped(const Gemm* qs, int count, hipStream_t stream, Workspace* ws = nullptr,
                  GemmPrec prec = GemmPrec::F64);

// Helpers for the common row-major cases.
inline Gemm gemm_nn(int M, int N, int K, const double* A, long lda, const double* B, long ldb, double* C,
                    long ldc, double alpha = 1.0, double beta = 0.0) {
  Gemm g; g.M = M; g.N = N; g.K = K;
  g.A = A; g.am = lda; g.ak = 1;
  g.B = B; g.bk = ldb; g.bn = 1;
  g.C = C; g.cm = ldc; g.cn = 1;
  g.alpha = alpha; g.beta = beta;
  return g;
}

}  // namespace ttipm
