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
#include "xlane.hpp"

namespace ttipm {

constexpr int BT = 1024;

constexpr int kTriMax = 32;

// Cholesky of an n x n (n <= 32) diagonal block (row-major, leading dimension
// lda), in place (lower), staged through LDS so that the n dependent steps do
// not wait on global memory.
__global__ __launch_bounds__(BT) void chol_block_kernel(double* A, int n, long lda, int* status, int offset) {
  __shared__ double As[kTriMax][kTriMax + 1];
  __shared__ int s_bad;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) As[t / n][t % n] = A[(long)(t / n) * lda + t % n];
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = As[j][j];
    if (!(d > 0.0)) {
      if (threadIdx.x == 0 && status[0] == 0) status[0] = offset + j + 1;
      s_bad = 1;
      break;
    }
    __syncthreads();   // every thread has read As[j][j]
    if (threadIdx.x == 0 || j + 1 + (int)threadIdx.x < n) {   // the threads that use the root
      const double dj = sqrt(d);
      if (threadIdx.x == 0) As[j][j] = dj;
      for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) As[i][j] /= dj;
    }
    __syncthreads();
    {   // thread (t / 32, t % 32) updates entry (j + 1 + t / 32, j + 1 + t % 32)
      const int i = j + 1 + (int)(threadIdx.x >> 5), c = j + 1 + (int)(threadIdx.x & 31);
      if (i < n && c <= i) As[i][c] -= As[i][j] * As[c][j];
    }
    __syncthreads();
  }
  if (s_bad) return;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, c = t % n;
    if (c <= i) A[(long)i * lda + c] = As[i][c];
  }
}

// Inverses of the n x n (n <= 32) diagonal blocks: one wave, one lane per
// column of the inverse.  The block is staged in LDS (every lane reads the same
// entry at a time: a broadcast) and each lane keeps its column in registers,
// so the substitution is a chain of FMAs with no memory round trips.

// lower triangular L (unit diagonal if unit != 0): forward substitution
__global__ __launch_bounds__(64) void trinv_lower_kernel(const double* L, int n, long lda, double* out, int unit) {
  __shared__ double Ls[kTriMax][kTriMax + 1];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) Ls[t / n][t % n] = L[(long)(t / n) * lda + t % n];
  __syncthreads();
  const int c = threadIdx.x;
  double x[kTriMax];
#pragma unroll
  for (int i = 0; i < kTriMax; ++i) {
    double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < i; ++j) acc -= Ls[i][j] * x[j];
    x[i] = (i < n) ? (unit ? acc : acc / Ls[i][i]) : 0.0;
  }
  if (c < n)
#pragma unroll
    for (int i = 0; i < kTriMax; ++i)
      if (i < n) out[(long)i * n + c] = x[i];
}

// upper triangular U: back substitution
__global__ __launch_bounds__(64) void trinv_upper_kernel(const double* U, int n, long lda, double* out) {
  __shared__ double Us[kTriMax][kTriMax + 1];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) Us[t / n][t % n] = U[(long)(t / n) * lda + t % n];
  __syncthreads();
  const int c = threadIdx.x;
  double x[kTriMax];
#pragma unroll
  for (int i = kTriMax - 1; i >= 0; --i) {
    double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = i + 1; j < kTriMax; ++j) acc -= (j < n ? Us[i][j] : 0.0) * x[j];
    x[i] = (i < n) ? acc / Us[i][i] : 0.0;
  }
  if (c < n)
#pragma unroll
    for (int i = 0; i < kTriMax; ++i)
      if (i < n) out[(long)i * n + c] = x[i];
}

// LU with partial pivoting of an m x nb panel (rows of a larger row-major
// matrix with leading dimension lda).  Row swaps are applied inside the panel;
// piv[t] receives the absolute row chosen at step t (row_base + local index).
__global__ __launch_bounds__(BT) void panel_lu_kernel(double* A, int m, int nb, long lda, int* piv, int row_base,
                                                      int* status) {
  __shared__ double rv[BT / 64];
  __shared__ int ri[BT / 64];
  for (int j = 0; j < nb && j < m; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < m; i += blockDim.x) {
      double v = fabs(A[(long)i * lda + j]);
      if (v > best) { best = v; bi = i; }
    }
    xlane::block_argmax<BT / 64>(best, bi, min(BT / 64, (m - j + 63) / 64), rv, ri);
    if (threadIdx.x == 0) piv[j] = row_base + bi;
    const int p = bi;
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
    {   // thread t updates column j + 1 + t % 32 of rows j + 1 + t / 32 + 32 k (nb <= 32)
      const int c = j + 1 + (int)(threadIdx.x & 31);
      if (c < nb)
        for (int i = j + 1 + (int)(threadIdx.x >> 5); i < m; i += BT / 32)
          A[(long)i * lda + c] -= A[(long)i * lda + j] * A[(long)j * lda + c];
    }
    __syncthreads();
  }
}

// The same panel factorisation with the panel staged in LDS (row stride
// nb + 1): for panels of up to a few hundred rows, where every step of the
// global-memory version waits on L2 latency.
__global__ __launch_bounds__(BT) void panel_lu_lds_kernel(double* A, int m, int nb, long lda, int* piv, int row_base,
                                                          int* status) {
  extern __shared__ double P[];
  __shared__ double rv[BT / 64];
  __shared__ int ri[BT / 64];
  const int ld = nb + 1;
  const int tid = threadIdx.x;
  for (int t = tid; t < m * nb; t += BT) P[(t / nb) * ld + t % nb] = A[(long)(t / nb) * lda + t % nb];
  __syncthreads();
  for (int j = 0; j < nb && j < m; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < m; i += BT) {
      const double v = fabs(P[i * ld + j]);
      if (v > best) { best = v; bi = i; }
    }
    xlane::block_argmax<BT / 64>(best, bi, min(BT / 64, (m - j + 63) / 64), rv, ri);
    if (tid == 0) piv[j] = row_base + bi;
    const int pv = bi;
    if (pv != j)
      for (int c = tid; c < nb; c += BT) {
        const double t = P[j * ld + c];
        P[j * ld + c] = P[pv * ld + c];
        P[pv * ld + c] = t;
      }
    __syncthreads();
    const double d = P[j * ld + j];
    if (d == 0.0) {
      if (tid == 0 && status[0] == 0) status[0] = row_base + j + 1;
      __syncthreads();
      continue;
    }
    for (int i = j + 1 + tid; i < m; i += BT) P[i * ld + j] /= d;
    __syncthreads();
    {   // thread t updates column j + 1 + t % 32 of rows j + 1 + t / 32 + 32 k (nb <= 32)
      const int c = j + 1 + (tid & 31);
      if (c < nb)
        for (int i = j + 1 + (tid >> 5); i < m; i += BT / 32) P[i * ld + c] -= P[i * ld + j] * P[j * ld + c];
    }
    __syncthreads();
  }
  for (int t = tid; t < m * nb; t += BT) A[(long)(t / nb) * lda + t % nb] = P[(t / nb) * ld + t % nb];
}

// Dynamic LDS available to the LDS panel kernel (device limit minus its
// static reduction arrays), opted in above the 64 KiB default.
static size_t panel_lds_limit() {
  static size_t limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
      (void)hipGetLastError();
      return (size_t)0;
    }
    size_t lim = (size_t)v - (size_t)BT * 12 - 256;
    if (lim > 65536 - (size_t)BT * 12 - 256 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&panel_lu_lds_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess) {
      (void)hipGetLastError();
      lim = 65536 - (size_t)BT * 12 - 256;
    }
    return lim;
  }();
  return limit;
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
// host drivers: recursive (divide and conquer) formulations.  Splitting the
// range in two halves at a multiple of nb turns the updates into GEMMs whose
// inner dimension is half the range, instead of nb-wide rank updates that
// rewrite the trailing matrix n / nb times.  Leaves are the nb x nb diagonal
// blocks (factorised and inverted by one workgroup) or the nb-wide LU panels.
// ---------------------------------------------------------------------------
namespace {

int split_at(int len, int nb) {
  int h = ((len / 2 + nb - 1) / nb) * nb;
  return (h >= len) ? len - nb : h;
}

const double* dblock(const DevBuf& d, int j0, int nb) { return d.get() + (size_t)(j0 / nb) * nb * nb; }

// op(L) X = B for rows [j0, j0+len) of B (ldb), L lower (ldl) with inverted
// diagonal blocks dinv (block j0/nb, stride = its size).  trans: L^T X = B.
void trsm_left_rec(const double* L, long ldl, const DevBuf& dinv, int nb, int j0, int len, double* B, long ldb,
                   int nrhs, bool trans, DevBuf& tmp, Ctx& c) {
  if (len <= nb) {
    const double* D = dblock(dinv, j0, nb);
    tmp.reserve((size_t)len * nrhs);
    double* Bj = B + (long)j0 * ldb;
    Gemm g;   // X = op(D) B_j
    g.M = len; g.N = nrhs; g.K = len;
    g.A = D; g.am = trans ? 1 : len; g.ak = trans ? len : 1;
    g.B = Bj; g.bk = ldb; g.bn = 1;
    g.C = tmp.get(); g.cm = nrhs; g.cn = 1;
    gemm(g, c.s, &c.ws, GemmPrec::F64);
    copy2d(tmp.get(), nrhs, Bj, ldb, len, nrhs, c.s);
    return;
  }
  const int h = split_at(len, nb);
  if (!trans) {
    trsm_left_rec(L, ldl, dinv, nb, j0, h, B, ldb, nrhs, trans, tmp, c);
    // B2 -= L21 X1
    gemm(gemm_nn(len - h, nrhs, h, L + (long)(j0 + h) * ldl + j0, ldl, B + (long)j0 * ldb, ldb,
                 B + (long)(j0 + h) * ldb, ldb, -1.0, 1.0),
         c.s, &c.ws, GemmPrec::F64);
    trsm_left_rec(L, ldl, dinv, nb, j0 + h, len - h, B, ldb, nrhs, trans, tmp, c);
  } else {
    trsm_left_rec(L, ldl, dinv, nb, j0 + h, len - h, B, ldb, nrhs, trans, tmp, c);
    Gemm u;   // B1 -= L21^T X2
    u.M = h; u.N = nrhs; u.K = len - h;
    u.A = L + (long)(j0 + h) * ldl + j0; u.am = 1; u.ak = ldl;
    u.B = B + (long)(j0 + h) * ldb; u.bk = ldb; u.bn = 1;
    u.C = B + (long)j0 * ldb; u.cm = ldb; u.cn = 1;
    u.alpha = -1.0; u.beta = 1.0;
    gemm(u, c.s, &c.ws, GemmPrec::F64);
    trsm_left_rec(L, ldl, dinv, nb, j0, h, B, ldb, nrhs, trans, tmp, c);
  }
}

// U X = B for rows [j0, j0+len) of B, U upper (ldu) with inverted diagonal blocks uinv.
void trsm_upper_rec(const double* U, long ldu, const DevBuf& uinv, int nb, int j0, int len, double* B, long ldb,
                    int nrhs, DevBuf& tmp, Ctx& c) {
  if (len <= nb) {
    const double* D = dblock(uinv, j0, nb);
    tmp.reserve((size_t)len * nrhs);
    double* Bj = B + (long)j0 * ldb;
    gemm(gemm_nn(len, nrhs, len, D, len, Bj, ldb, tmp.get(), nrhs), c.s, &c.ws, GemmPrec::F64);
    copy2d(tmp.get(), nrhs, Bj, ldb, len, nrhs, c.s);
    return;
  }
  const int h = split_at(len, nb);
  trsm_upper_rec(U, ldu, uinv, nb, j0 + h, len - h, B, ldb, nrhs, tmp, c);
  // B1 -= U12 X2
  gemm(gemm_nn(h, nrhs, len - h, U + (long)j0 * ldu + (j0 + h), ldu, B + (long)(j0 + h) * ldb, ldb,
               B + (long)j0 * ldb, ldb, -1.0, 1.0),
       c.s, &c.ws, GemmPrec::F64);
  trsm_upper_rec(U, ldu, uinv, nb, j0, h, B, ldb, nrhs, tmp, c);
}

// X L^T = B (right side) for the diagonal range [j0, j0+len) of L; B is m x len (ldb),
// its column q corresponds to L's row/column j0 + q.
void trsm_right_lt_rec(const double* L, long ldl, const DevBuf& dinv, int nb, int j0, int len, double* B, long ldb,
                       int m, DevBuf& tmp, Ctx& c) {
  if (len <= nb) {
    const double* D = dblock(dinv, j0, nb);
    tmp.reserve((size_t)m * len);
    Gemm g;   // X = B D^T
    g.M = m; g.N = len; g.K = len;
    g.A = B; g.am = ldb; g.ak = 1;
    g.B = D; g.bk = 1; g.bn = len;
    g.C = tmp.get(); g.cm = len; g.cn = 1;
    gemm(g, c.s, &c.ws, GemmPrec::F64);
    copy2d(tmp.get(), len, B, ldb, m, len, c.s);
    return;
  }
  const int h = split_at(len, nb);
  trsm_right_lt_rec(L, ldl, dinv, nb, j0, h, B, ldb, m, tmp, c);
  Gemm u;   // B2 -= X1 L21^T
  u.M = m; u.N = len - h; u.K = h;
  u.A = B; u.am = ldb; u.ak = 1;
  u.B = L + (long)(j0 + h) * ldl + j0; u.bk = 1; u.bn = ldl;
  u.C = B + h; u.cm = ldb; u.cn = 1;
  u.alpha = -1.0; u.beta = 1.0;
  gemm(u, c.s, &c.ws, GemmPrec::F64);
  trsm_right_lt_rec(L, ldl, dinv, nb, j0 + h, len - h, B + h, ldb, m, tmp, c);
}

void chol_rec(double* A, int n, BlockedFactors& f, int j0, int len, int* st, DevBuf& tmp, Ctx& c) {
  const int nb = f.nb;
  if (len <= nb) {
    double* Ajj = A + (long)j0 * n + j0;
    TT_REQUIRE(len <= kTriMax, "diagonal block above 32");
    hipLaunchKernelGGL(chol_block_kernel, dim3(1), dim3(BT), 0, c.s, Ajj, len, (long)n, st, j0);
    hipLaunchKernelGGL(trinv_lower_kernel, dim3(1), dim3(64), 0, c.s, Ajj, len, (long)n,
                       const_cast<double*>(dblock(f.dinv, j0, nb)), 0);
    TT_HIP(hipGetLastError());
    return;
  }
  const int h = split_at(len, nb);
  chol_rec(A, n, f, j0, h, st, tmp, c);
  // L21 = A21 L11^{-T}
  double* A21 = A + (long)(j0 + h) * n + j0;
  trsm_right_lt_rec(A, n, f.dinv, nb, j0, h, A21, n, len - h, tmp, c);
  // A22 -= L21 L21^T
  Gemm u;
  u.M = len - h; u.N = len - h; u.K = h;
  u.A = A21; u.am = n; u.ak = 1;
  u.B = A21; u.bk = 1; u.bn = n;
  u.C = A + (long)(j0 + h) * n + (j0 + h); u.cm = n; u.cn = 1;
  u.alpha = -1.0; u.beta = 1.0;
  gemm(u, c.s, &c.ws, GemmPrec::F64);
  chol_rec(A, n, f, j0 + h, len - h, st, tmp, c);
}

// LU of the columns [j0, j0+w) over rows [j0, n), rows swapped inside these
// columns only (the caller swaps the other columns).
void lu_rec(double* A, int n, BlockedFactors& f, int* piv, int j0, int w, int* st, DevBuf& tmp, Ctx& c) {
  const int nb = f.nb;
  if (w <= nb) {
    TT_REQUIRE(w <= kTriMax, "diagonal block above 32");   // the panel kernels take at most 32 columns
    const double pm = n - j0;
    const size_t lds = sizeof(double) * (size_t)(n - j0) * (w + 1);
    if (lds <= panel_lds_limit())
      launch_prof(PK_PANEL_LU, pm * w * (double)w, 16.0 * pm * w, panel_lu_lds_kernel, dim3(1), dim3(BT),
                  (unsigned)lds, c.s, A + (long)j0 * n + j0, n - j0, w, (long)n, piv + j0, j0, st);
    else
      launch_prof(PK_PANEL_LU, pm * w * (double)w, 16.0 * pm * w, panel_lu_kernel, dim3(1), dim3(BT), 0, c.s,
                  A + (long)j0 * n + j0, n - j0, w, (long)n, piv + j0, j0, st);
    double* Ajj = A + (long)j0 * n + j0;
    hipLaunchKernelGGL(trinv_lower_kernel, dim3(1), dim3(64), 0, c.s, Ajj, w, (long)n,
                       const_cast<double*>(dblock(f.dinv, j0, nb)), 1);
    hipLaunchKernelGGL(trinv_upper_kernel, dim3(1), dim3(64), 0, c.s, Ajj, w, (long)n,
                       const_cast<double*>(dblock(f.uinv, j0, nb)));
    TT_HIP(hipGetLastError());
    return;
  }
  const int h = split_at(w, nb);
  lu_rec(A, n, f, piv, j0, h, st, tmp, c);
  // the left half's row swaps on the right half's columns
  hipLaunchKernelGGL(apply_swaps_kernel, dim3(nblocks(w - h, 64)), dim3(64), 0, c.s, A, (long)n, piv + j0, j0, h,
                     j0 + h, j0 + w);
  TT_HIP(hipGetLastError());
  // A12 = L11^{-1} A12 (unit lower), A22 -= A21 A12
  double* A12 = A + (long)j0 * n + (j0 + h);
  trsm_left_rec(A, n, f.dinv, nb, j0, h, A + (j0 + h), n, w - h, false, tmp, c);
  gemm(gemm_nn(n - j0 - h, w - h, h, A + (long)(j0 + h) * n + j0, n, A12, n, A + (long)(j0 + h) * n + (j0 + h), n,
               -1.0, 1.0),
       c.s, &c.ws, GemmPrec::F64);
  lu_rec(A, n, f, piv, j0 + h, w - h, st, tmp, c);
  // the right half's row swaps on the left half's columns
  hipLaunchKernelGGL(apply_swaps_kernel, dim3(nblocks(h, 64)), dim3(64), 0, c.s, A, (long)n, piv + j0 + h, j0 + h,
                     w - h, j0, j0 + h);
  TT_HIP(hipGetLastError());
}

}  // namespace

int chol_blocked(double* A, int n, BlockedFactors& f, Ctx& c) {
  const int nb = f.nb;
  const int nblk = (n + nb - 1) / nb;
  f.n = n;
  f.dinv.reserve((size_t)nblk * nb * nb);
  c.ired.reserve(4);
  int* st = reinterpret_cast<int*>(c.ired.get());
  TT_HIP(hipMemsetAsync(st, 0, sizeof(int), c.s));
  DevBuf tmp;
  chol_rec(A, n, f, 0, n, st, tmp, c);
  int hst = 0;
  TT_HIP(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return hst;
}

void trsm_blocked(const double* L, int n, const BlockedFactors& f, double* B, int nrhs, bool trans, Ctx& c) {
  DevBuf tmp;
  trsm_left_rec(L, n, f.dinv, f.nb, 0, n, B, nrhs, nrhs, trans, tmp, c);
  // tmp goes back to this stream's free list: later work on the stream
  // reuses it only after these kernels
}

int lu_blocked(double* A, int n, BlockedFactors& f, Ctx& c) {
  const int nb = f.nb;
  const int nblk = (n + nb - 1) / nb;
  f.n = n;
  f.piv.reserve((size_t)n / 2 + 1);         // ints packed in doubles
  f.dinv.reserve((size_t)nblk * nb * nb);   // inverses of the unit-lower diagonal blocks
  f.uinv.reserve((size_t)nblk * nb * nb);   // inverses of the upper diagonal blocks
  int* piv = reinterpret_cast<int*>(f.piv.get());
  c.ired.reserve(4);
  int* st = reinterpret_cast<int*>(c.ired.get());
  TT_HIP(hipMemsetAsync(st, 0, sizeof(int), c.s));
  DevBuf tmp;
  lu_rec(A, n, f, piv, 0, n, st, tmp, c);
  int hst = 0;
  TT_HIP(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return hst;
}

void lu_solve_blocked(const double* A, int n, const BlockedFactors& f, double* B, int nrhs, Ctx& c) {
  const int* piv = reinterpret_cast<const int*>(f.piv.get());
  hipLaunchKernelGGL(permute_rhs_kernel, dim3(nblocks(nrhs, 64)), dim3(64), 0, c.s, B, n, nrhs, piv);
  TT_HIP(hipGetLastError());
  DevBuf tmp;
  // forward with the unit lower factor, then backward with the upper factor
  trsm_left_rec(A, n, f.dinv, f.nb, 0, n, B, nrhs, nrhs, false, tmp, c);
  trsm_upper_rec(A, n, f.uinv, f.nb, 0, n, B, nrhs, nrhs, tmp, c);
  c.sync();
}

}  // namespace ttipm
