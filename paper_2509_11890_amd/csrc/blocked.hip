// Blocked dense factorisations for the local direct solves of large frames.
//
// The block elimination of the reduced KKT system (Sec. 3.3) needs a Cholesky
// factorisation of L_Z^ (p x p), triangular solves with p right-hand sides and
// an LU factorisation of the Schur complement S.  For p in the thousands the
// right-looking blocked algorithms below put almost all flops into the MFMA
// GEMM (panel updates and trailing-matrix updates); only the nb x nb diagonal
// blocks and the p x nb LU panels are factorised by a single workgroup.
// Diagonal blocks are inverted explicitly so that the triangular solves with
// many right-hand sides are GEMMs as well.
#include "blocked.hpp"

#include <algorithm>
#include <cmath>

#include "ttops.hpp"

namespace ttipm {

constexpr int BT = 1024;

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Cholesky of an n x n diagonal block (row-major, leading dimension lda), in place (lower).
__global__ __launch_bounds__(BT) void chol_block_kernel(double* A, int n, long lda, int* status, int offset) {
  __shared__ double s_d;
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = A[(long)j * lda + j];
      if (!(d > 0.0)) {
        s_bad = 1;
        if (status[0] == 0) status[0] = offset + j + 1;
      }
      s_d = (d > 0.0) ? sqrt(d) : 1.0;
      A[(long)j * lda + j] = s_d;
    }
    __syncthreads();
    if (s_bad) return;
    const double dj = s_d;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[(long)i * lda + j] /= dj;
    __syncthreads();
    const int rows = n - j - 1;
    for (long t = threadIdx.x; t < (long)rows * rows; t += blockDim.x) {
      int i = j + 1 + (int)(t / rows), c = j + 1 + (int)(t % rows);
      if (c <= i) A[(long)i * lda + c] -= A[(long)i * lda + j] * A[(long)c * lda + j];
    }
    __syncthreads();
  }
}

// Inverse of a lower-triangular n x n block (unit diagonal if unit != 0):
// one thread per column solves L x = e_c by forward substitution.
__global__ void trinv_lower_kernel(const double* L, int n, long lda, double* out, int unit) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int i = 0; i < n; ++i) {
    if (i < c) {
      out[(long)i * n + c] = 0.0;
      continue;
    }
    double acc = (i == c) ? 1.0 : 0.0;
    for (int j = c; j < i; ++j) acc -= L[(long)i * lda + j] * out[(long)j * n + c];
    out[(long)i * n + c] = unit ? acc : acc / L[(long)i * lda + i];
  }
}

// Inverse of an upper-triangular n x n block: one thread per column, back substitution.
__global__ void trinv_upper_kernel(const double* U, int n, long lda, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int i = n - 1; i >= 0; --i) {
    if (i > c) {
      out[(long)i * n + c] = 0.0;
      continue;
    }
    double acc = (i == c) ? 1.0 : 0.0;
    for (int j = i + 1; j <= c; ++j) acc -= U[(long)i * lda + j] * out[(long)j * n + c];
    out[(long)i * n + c] = acc / U[(long)i * lda + i];
  }
}

// LU with partial pivoting of an m x nb panel (rows of a larger row-major
// matrix with leading dimension lda).  Row swaps are applied inside the panel;
// piv[t] receives the absolute row chosen at step t (row_base + local index).
__global__ __launch_bounds__(BT) void panel_lu_kernel(double* A, int m, int nb, long lda, int* piv, int row_base,
                                                      int* status) {
  __shared__ double rv[BT];
  __shared__ int ri[BT];
  __shared__ int s_piv;
  for (int j = 0; j < nb && j < m; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < m; i += blockDim.x) {
      double v = fabs(A[(long)i * lda + j]);
      if (v > best) { best = v; bi = i; }
    }
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        double a = rv[threadIdx.x], b = rv[threadIdx.x + o];
        int ia = ri[threadIdx.x], ib = ri[threadIdx.x + o];
        if (b > a || (b == a && ib < ia)) { rv[threadIdx.x] = b; ri[threadIdx.x] = ib; }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      s_piv = ri[0];
      piv[j] = row_base + ri[0];
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j)
      for (int c = threadIdx.x; c < nb; c += blockDim.x) {
        double t = A[(long)j * lda + c];
        A[(long)j * lda + c] = A[(long)p * lda + c];
        A[(long)p * lda + c] = t;
      }
    __syncthreads();
    const double d = A[(long)j * lda + j];
    if (d == 0.0) {
      if (threadIdx.x == 0 && status[0] == 0) status[0] = row_base + j + 1;
      __syncthreads();
      continue;
    }
    for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) A[(long)i * lda + j] /= d;
    __syncthreads();
    const int rows = m - j - 1, cols = nb - j - 1;
    for (long t = threadIdx.x; t < (long)rows * cols; t += blockDim.x) {
      int i = j + 1 + (int)(t / cols), c = j + 1 + (int)(t % cols);
      A[(long)i * lda + c] -= A[(long)i * lda + j] * A[(long)j * lda + c];
    }
    __syncthreads();
  }
}

// Apply the row swaps of one panel (rows j0 .. j0+nb-1 swapped with piv[t])
// to the columns [c0, c1): one thread per column, swaps in order.
__global__ void apply_swaps_kernel(double* A, long lda, const int* piv, int j0, int nb, int c0, int c1) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  for (int t = 0; t < nb; ++t) {
    const int r = j0 + t, p = piv[t];
    if (p != r) {
      double v = A[(long)r * lda + c];
      A[(long)r * lda + c] = A[(long)p * lda + c];
      A[(long)p * lda + c] = v;
    }
  }
}

// b <- P b for the recorded pivots (sequential), nrhs columns.
__global__ void permute_rhs_kernel(double* B, int n, int nrhs, const int* piv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  for (int r = 0; r < n; ++r) {
    const int p = piv[r];
    if (p != r) {
      double v = B[(long)r * nrhs + c];
      B[(long)r * nrhs + c] = B[(long)p * nrhs + c];
      B[(long)p * nrhs + c] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------
int chol_blocked(double* A, int n, BlockedFactors& f, Ctx& c) {
  const int nb = f.nb;
  const int nblk = (n + nb - 1) / nb;
  f.n = n;
  f.dinv.reserve((size_t)nblk * nb * nb);
  c.ired.reserve(4);
  int* st = reinterpret_cast<int*>(c.ired.get());
  TT_HIP(hipMemsetAsync(st, 0, sizeof(int), c.s));
  DevBuf T((size_t)n * nb);
  for (int j = 0; j < n; j += nb) {
    const int jb = std::min(nb, n - j);
    double* Ajj = A + (long)j * n + j;
    hipLaunchKernelGGL(chol_block_kernel, dim3(1), dim3(BT), 0, c.s, Ajj, jb, (long)n, st, j);
    double* Dj = f.dinv.get() + (size_t)(j / nb) * nb * nb;
    hipLaunchKernelGGL(trinv_lower_kernel, dim3(1), dim3(std::max(64, ((jb + 63) / 64) * 64)), 0, c.s, Ajj, jb,
                       (long)n, Dj, 0);
    TT_HIP(hipGetLastError());
    const int rest = n - j - jb;
    if (rest > 0) {
      // panel <- panel L_jj^{-T}
      double* Pn = A + (long)(j + jb) * n + j;
      Gemm g;
      g.M = rest; g.N = jb; g.K = jb;
      g.A = Pn; g.am = n; g.ak = 1;
      g.B = Dj; g.bk = 1; g.bn = jb;          // (L^{-1})^T [k][c] = L^{-1}[c][k]
      g.C = T.get(); g.cm = jb; g.cn = 1;
      gemm(g, c.s, &c.ws, GemmPrec::F64);
      copy2d(T.get(), jb, Pn, n, rest, jb, c.s);
      // trailing A22 -= P P^T
      Gemm u;
      u.M = rest; u.N = rest; u.K = jb;
      u.A = Pn; u.am = n; u.ak = 1;
      u.B = Pn; u.bk = 1; u.bn = n;
      u.C = A + (long)(j + jb) * n + (j + jb); u.cm = n; u.cn = 1;
      u.alpha = -1.0; u.beta = 1.0;
      gemm(u, c.s, &c.ws, GemmPrec::F64);
    }
  }
  int hst = 0;
  TT_HIP(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return hst;
}

void trsm_blocked(const double* L, int n, const BlockedFactors& f, double* B, int nrhs, bool trans, Ctx& c) {
  const int nb = f.nb;
  DevBuf X((size_t)nb * nrhs);
  if (!trans) {
    for (int j = 0; j < n; j += nb) {
      const int jb = std::min(nb, n - j);
      const double* Dj = f.dinv.get() + (size_t)(j / nb) * nb * nb;
      double* Bj = B + (long)j * nrhs;
      gemm(gemm_nn(jb, nrhs, jb, Dj, jb, Bj, nrhs, X.get(), nrhs), c.s, &c.ws, GemmPrec::F64);
      TT_HIP(hipMemcpyAsync(Bj, X.get(), sizeof(double) * (size_t)jb * nrhs, hipMemcpyDeviceToDevice, c.s));
      const int rest = n - j - jb;
      if (rest > 0)
        gemm(gemm_nn(rest, nrhs, jb, L + (long)(j + jb) * n + j, n, X.get(), nrhs, B + (long)(j + jb) * nrhs, nrhs,
                     -1.0, 1.0),
             c.s, &c.ws, GemmPrec::F64);
    }
  } else {
    const int nblk = (n + nb - 1) / nb;
    for (int bj = nblk - 1; bj >= 0; --bj) {
      const int j = bj * nb;
      const int jb = std::min(nb, n - j);
      const double* Dj = f.dinv.get() + (size_t)bj * nb * nb;
      double* Bj = B + (long)j * nrhs;
      Gemm g;   // X = D_j^T B_j
      g.M = jb; g.N = nrhs; g.K = jb;
      g.A = Dj; g.am = 1; g.ak = jb;
      g.B = Bj; g.bk = nrhs; g.bn = 1;
      g.C = X.get(); g.cm = nrhs; g.cn = 1;
      gemm(g, c.s, &c.ws, GemmPrec::F64);
      TT_HIP(hipMemcpyAsync(Bj, X.get(), sizeof(double) * (size_t)jb * nrhs, hipMemcpyDeviceToDevice, c.s));
      if (j > 0) {
        Gemm u;   // B[0:j] -= L[j:j+jb, 0:j]^T X
        u.M = j; u.N = nrhs; u.K = jb;
        u.A = L + (long)j * n; u.am = 1; u.ak = n;
        u.B = X.get(); u.bk = nrhs; u.bn = 1;
        u.C = B; u.cm = nrhs; u.cn = 1;
        u.alpha = -1.0; u.beta = 1.0;
        gemm(u, c.s, &c.ws, GemmPrec::F64);
      }
    }
  }
}

int lu_blocked(double* A, int n, BlockedFactors& f, Ctx& c) {
  const int nb = f.nb;
  const int nblk = (n + nb - 1) / nb;
  f.n = n;
  f.piv.reserve((size_t)n / 2 + 1);     // ints packed in doubles
  f.dinv.reserve((size_t)nblk * nb * nb);   // inverses of the unit-lower diagonal blocks
  f.uinv.reserve((size_t)nblk * nb * nb);   // inverses of the upper diagonal blocks
  int* piv = reinterpret_cast<int*>(f.piv.get());
  c.ired.reserve(4);
  int* st = reinterpret_cast<int*>(c.ired.get());
  TT_HIP(hipMemsetAsync(st, 0, sizeof(int), c.s));
  DevBuf T((size_t)nb * n);
  for (int j = 0; j < n; j += nb) {
    const int jb = std::min(nb, n - j);
    const double pm = n - j;
    const int tok = prof_begin(PK_PANEL_LU, c.s, pm * jb * (double)jb, 16.0 * pm * jb);
    hipLaunchKernelGGL(panel_lu_kernel, dim3(1), dim3(BT), 0, c.s, A + (long)j * n + j, n - j, jb, (long)n, piv + j, j,
                       st);
    prof_end(tok, c.s);
    TT_HIP(hipGetLastError());
    // panel pivots are relative to the panel's first row: convert to absolute rows
    // (the kernel already adds row_base), then swap rows outside the panel columns
    if (j > 0)
      hipLaunchKernelGGL(apply_swaps_kernel, dim3(nblocks(j, 256)), dim3(256), 0, c.s, A, (long)n, piv + j, j, jb, 0, j);
    if (j + jb < n)
      hipLaunchKernelGGL(apply_swaps_kernel, dim3(nblocks(n - j - jb, 256)), dim3(256), 0, c.s, A, (long)n, piv + j, j,
                         jb, j + jb, n);
    TT_HIP(hipGetLastError());
    double* Ajj = A + (long)j * n + j;
    double* Dj = f.dinv.get() + (size_t)(j / nb) * nb * nb;
    double* Uj = f.uinv.get() + (size_t)(j / nb) * nb * nb;
    const unsigned tb = std::max(64, ((jb + 63) / 64) * 64);
    hipLaunchKernelGGL(trinv_lower_kernel, dim3(1), dim3(tb), 0, c.s, Ajj, jb, (long)n, Dj, 1);
    hipLaunchKernelGGL(trinv_upper_kernel, dim3(1), dim3(tb), 0, c.s, Ajj, jb, (long)n, Uj);
    TT_HIP(hipGetLastError());
    const int rest = n - j - jb;
    if (rest > 0) {
      // U12 = L11^{-1} A12
      double* A12 = A + (long)j * n + (j + jb);
      gemm(gemm_nn(jb, rest, jb, Dj, jb, A12, n, T.get(), rest), c.s, &c.ws, GemmPrec::F64);
      copy2d(T.get(), rest, A12, n, jb, rest, c.s);
      // A22 -= L21 U12
      gemm(gemm_nn(rest, rest, jb, A + (long)(j + jb) * n + j, n, A12, n, A + (long)(j + jb) * n + (j + jb), n, -1.0,
                   1.0),
           c.s, &c.ws, GemmPrec::F64);
    }
  }
  int hst = 0;
  TT_HIP(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return hst;
}

void lu_solve_blocked(const double* A, int n, const BlockedFactors& f, double* B, int nrhs, Ctx& c) {
  const int nb = f.nb;
  const int* piv = reinterpret_cast<const int*>(f.piv.get());
  hipLaunchKernelGGL(permute_rhs_kernel, dim3(nblocks(nrhs, 64)), dim3(64), 0, c.s, B, n, nrhs, piv);
  TT_HIP(hipGetLastError());
  DevBuf X((size_t)nb * nrhs);
  // forward: unit lower
  for (int j = 0; j < n; j += nb) {
    const int jb = std::min(nb, n - j);
    const double* Dj = f.dinv.get() + (size_t)(j / nb) * nb * nb;
    double* Bj = B + (long)j * nrhs;
    gemm(gemm_nn(jb, nrhs, jb, Dj, jb, Bj, nrhs, X.get(), nrhs), c.s, &c.ws, GemmPrec::F64);
    TT_HIP(hipMemcpyAsync(Bj, X.get(), sizeof(double) * (size_t)jb * nrhs, hipMemcpyDeviceToDevice, c.s));
    const int rest = n - j - jb;
    if (rest > 0)
      gemm(gemm_nn(rest, nrhs, jb, A + (long)(j + jb) * n + j, n, X.get(), nrhs, B + (long)(j + jb) * nrhs, nrhs, -1.0,
                   1.0),
           c.s, &c.ws, GemmPrec::F64);
  }
  // backward: upper
  const int nblk = (n + nb - 1) / nb;
  for (int bj = nblk - 1; bj >= 0; --bj) {
    const int j = bj * nb;
    const int jb = std::min(nb, n - j);
    const double* Uj = f.uinv.get() + (size_t)bj * nb * nb;
    double* Bj = B + (long)j * nrhs;
    gemm(gemm_nn(jb, nrhs, jb, Uj, jb, Bj, nrhs, X.get(), nrhs), c.s, &c.ws, GemmPrec::F64);
    TT_HIP(hipMemcpyAsync(Bj, X.get(), sizeof(double) * (size_t)jb * nrhs, hipMemcpyDeviceToDevice, c.s));
    if (j > 0)
      gemm(gemm_nn(j, nrhs, jb, A + j, n, X.get(), nrhs, B, nrhs, -1.0, 1.0), c.s, &c.ws, GemmPrec::F64);
  }
}

}  // namespace ttipm
