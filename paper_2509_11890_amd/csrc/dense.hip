// Small dense FP64 factorisations that stay on the device: Householder QR,
// one-sided Jacobi SVD, LU with partial pivoting, Cholesky and triangular
// solves.  They serve TT rounding (QR + truncated SVD, Sec. 2.3), the SVD move
// of the block index in AMEn (Sec. 2.3, Block TT), the dense local solve
// (Sec. 3.3) and the generalised eigenproblems of the step length (Sec. 3.4).
//
// The matrices are small (at most a few thousand rows, a few hundred columns),
// so each factorisation runs in one 1024-thread workgroup: the matrix lives in
// global memory (resident in the XCD's L2), columns are processed with 64-lane
// wavefront reductions, and the workgroup synchronises between the sequential
// steps of the algorithm.  Reductions use a fixed order, so results are
// reproducible run to run.
#include "dense.hpp"
#include "xlane.hpp"

#include <algorithm>
#include <cmath>

namespace ttipm {

constexpr int DT = 1024;        // threads per dense workgroup
constexpr int NW = DT / 64;     // waves per workgroup

__device__ __forceinline__ double wave_sum(double v) { return xlane::wave_sum(v); }

// Block-wide sum of nonnegative partials (sums of squares) over a workgroup of
// DT threads with a fixed reduction order (result broadcast to all threads).
// Only the first `active` threads may hold nonzero partials: the wavefronts
// beyond them hold +0 and are left out, which leaves the sum unchanged, and
// do no reduction work (they share the SIMDs with the ones that do).
__device__ double block_sum(double v, double* red, int active = DT) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int nwa = min(NW, (active + 63) / 64);
  if (w < nwa) v = wave_sum(v);
  __syncthreads();
  if (lane == 0 && w < nwa) red[w] = v;
  __syncthreads();
  double r[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i)
    if (i < nwa) r[i] = red[i];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i)
    if (i < nwa) s += r[i];
  __syncthreads();
  return s;
}

// v_j^T x over the rows j + lane, j + lane + 64, ... < m of one lane (v_j[j] = 1
// implicit), summed in that order; four loads per operand are issued before
// the first product waits on them.
__device__ __forceinline__ double reflector_dot(const double* v, const double* x, int j, int m, int lane) {
  double d = 0.0;
  for (int i0 = j + lane; i0 < m; i0 += 256) {
    double vs[4], xs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u;
      vs[u] = i < m ? ((i == j) ? 1.0 : v[i]) : 0.0;
      xs[u] = i < m ? x[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 64 * u < m) d += vs[u] * xs[u];
  }
  return d;
}

// x -= d v_j over the rows of one lane (v_j[j] = 1 implicit), four rows at a
// time with their loads issued first.
__device__ __forceinline__ void reflector_update(const double* v, double* x, int j, int m, int lane, double d) {
  for (int i0 = j + lane; i0 < m; i0 += 256) {
    double vs[4], xs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u;
      vs[u] = i < m ? ((i == j) ? 1.0 : v[i]) : 0.0;
      xs[u] = i < m ? x[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 64 * u < m) x[i0 + 64 * u] = xs[u] - d * vs[u];
  }
}

// ---------------------------------------------------------------------------
// Householder QR, column-major A (m x n, leading dimension lda), in place.
// On exit R is in the upper triangle, the reflector vectors v_j (v_j[j] = 1
// implicit) below it, and tau[j] their scalars: H_j = I - tau_j v_j v_j^T.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(DT) void qr_kernel(double* A, int m, int n, int lda, double* tau) {
  __shared__ double red[NW];
  __shared__ double s_beta, s_tau, s_scale;
  const int kmax = min(m, n);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  for (int j = 0; j < kmax; ++j) {
    double* col = A + (long)j * lda;
    double part = 0.0;
    for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) part += col[i] * col[i];
    double sig = block_sum(part, red, m - j - 1);
    if (threadIdx.x == 0) {
      double alpha = col[j];
      if (sig == 0.0) {
        s_tau = 0.0; s_beta = alpha; s_scale = 0.0;
      } else {
        double nrm = sqrt(alpha * alpha + sig);
        double beta = (alpha <= 0.0) ? nrm : -nrm;
        s_tau = (beta - alpha) / beta;
        s_scale = 1.0 / (alpha - beta);
        s_beta = beta;
      }
      tau[j] = s_tau;
    }
    __syncthreads();
    const double sc = s_scale, tj = s_tau;
    for (int i = j + 1 + threadIdx.x; i < m; i += blockDim.x) col[i] *= sc;
    __syncthreads();
    if (threadIdx.x == 0) col[j] = s_beta;
    // apply H_j to trailing columns: one wave per column
    if (tj != 0.0) {
      for (int c = j + 1 + w; c < n; c += NW) {
        double* cc = A + (long)c * lda;
        double d = wave_sum(reflector_dot(col, cc, j, m, lane)) * tj;
        reflector_update(col, cc, j, m, lane, d);
      }
    }
    __syncthreads();
  }
}

// Explicit Q (m x k, column-major, ldq) from the reflectors: Q = H_0 ... H_{k-1} I.
__global__ __launch_bounds__(DT) void qr_form_q_kernel(const double* A, int m, int n, int lda,
                                                       const double* tau, double* Q, int k, int ldq) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  for (long t = threadIdx.x; t < (long)m * k; t += blockDim.x) {
    int c = (int)(t / m), i = (int)(t % m);
    Q[(long)c * ldq + i] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kmax = min(min(m, n), k);
  for (int j = kmax - 1; j >= 0; --j) {
    const double* v = A + (long)j * lda;
    const double tj = tau[j];
    // columns c < j are still e_c, which H_j leaves unchanged
    if (tj != 0.0) {
      for (int c = j + w; c < k; c += NW) {
        double* qc = Q + (long)c * ldq;
        double d = wave_sum(reflector_dot(v, qc, j, m, lane)) * tj;
        reflector_update(v, qc, j, m, lane, d);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of a column-major m x n matrix A (lda = m).
// Column pairs are rotated in the round-robin (tournament) order, n/2 disjoint
// pairs per step, one wavefront per pair.  On exit U (m x n, column-major),
// sigma (descending) and V (n x n, column-major) with A = U diag(sigma) V^T.
// Columns of U with sigma = 0 are zero.  work: m*n + n*n doubles + n ints.
// With Vw == nullptr the rotations are not accumulated and V is not written:
// the left singular vectors and the singular values alone (n <= 4096).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void jacobi_svd_body(double* A, int m, int n, double* Vw, double* U, double* sigma,
                                                double* V, int* order, int max_sweeps, double tol, int* sweeps_out,
                                                int* s_rot) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const bool wantv = Vw != nullptr;
  const double big = sqrt(tol);
  if (wantv)
    for (long t = threadIdx.x; t < (long)n * n; t += blockDim.x) {
      int c = (int)(t / n), i = (int)(t % n);
      Vw[t] = (i == c) ? 1.0 : 0.0;
    }
  __syncthreads();
  const int N = (n % 2) ? n + 1 : n;   // players incl. a dummy when n is odd
  // 16-lane groups rotate one column pair each (64 pairs in flight per step);
  // a group is active or idle as a whole, so its shuffles stay inside it.
  const int gl = threadIdx.x % 16, gid = threadIdx.x / 16;
  const int NG = blockDim.x / 16, nw = blockDim.x / 64;
  int sweep = 0;
  for (; sweep < max_sweeps && N > 1; ++sweep) {
    if (threadIdx.x == 0) { s_rot[0] = 0; s_rot[1] = 0; }
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      for (int pi = gid; pi < N / 2; pi += NG) {
        int p, q;
        if (pi == 0) { p = N - 1; q = r; }
        else { p = (r + pi) % (N - 1); q = (r - pi + N - 1) % (N - 1); }
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= n) continue;
        double* ap = A + (long)p * m;
        double* aq = A + (long)q * m;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < m; i += 16) {
          double x = ap[i], y = aq[i];
          al += x * x; be += y * y; ga += x * y;
        }
        al = xlane::row16_sum(al);
        be = xlane::row16_sum(be);
        ga = xlane::row16_sum(ga);
        if (ga == 0.0 || al == 0.0 || be == 0.0) continue;
        if (fabs(ga) <= tol * sqrt(al * be)) continue;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = gl; i < m; i += 16) {
          double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        if (wantv) {
          double* vp = Vw + (long)p * n;
          double* vq = Vw + (long)q * n;
          for (int i = gl; i < n; i += 16) {
            double x = vp[i], y = vq[i];
            vp[i] = c * x - s * y;
            vq[i] = s * x + c * y;
          }
        }
        if (gl == 0) {
          s_rot[0] = 1;
          if (fabs(ga) > big * sqrt(al * be)) s_rot[1] = 1;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    // Stop after a sweep without rotations, or one whose rotations were all
    // below sqrt(tol): convergence is quadratic, so the next sweep would find
    // every pair orthogonal to about tol and rotate none.
    if (!s_rot[0]) { ++sweep; break; }
    if (!s_rot[1]) { ++sweep; break; }
    __syncthreads();
  }
  // column norms
  for (int c = w; c < n; c += nw) {
    const double* ac = A + (long)c * m;
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += ac[i] * ac[i];
    s = wave_sum(s);
    if (lane == 0) sigma[c] = sqrt(s);   // unsorted for now
  }
  __syncthreads();
  // rank sort (descending, ties by index) -> order[rank] = column
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double sc = sigma[c];
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      double so = sigma[o];
      rank += (so > sc) || (so == sc && o < c);
    }
    order[rank] = c;
  }
  __syncthreads();
  for (long t = threadIdx.x; t < (long)m * n; t += blockDim.x) {
    int rnk = (int)(t / m), i = (int)(t % m);
    int c = order[rnk];
    double sc = sigma[c];
    U[t] = (sc > 0.0) ? A[(long)c * m + i] / sc : 0.0;
  }
  if (wantv)
    for (long t = threadIdx.x; t < (long)n * n; t += blockDim.x) {
      int rnk = (int)(t / n), i = (int)(t % n);
      V[t] = Vw[(long)order[rnk] * n + i];
    }
  // sigma in sorted order: gathered into registers, written back after a barrier
  double sv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int rnk = threadIdx.x + j * blockDim.x;
    sv[j] = (rnk < n) ? sigma[order[rnk]] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int rnk = threadIdx.x + j * blockDim.x;
    if (rnk < n) sigma[rnk] = sv[j];
  }
  if (threadIdx.x == 0 && sweeps_out) *sweeps_out = sweep;
}

__global__ __launch_bounds__(DT) void jacobi_svd_kernel(double* A, int m, int n, double* Vw, double* U,
                                                        double* sigma, double* V, int* order, int max_sweeps,
                                                        double tol, int* sweeps_out) {
  __shared__ int s_rot[2];
  jacobi_svd_body(A, m, n, Vw, U, sigma, V, order, max_sweeps, tol, sweeps_out, s_rot);
}

// The same sweeps with A and the rotation accumulator resident in LDS (dynamic
// shared memory of (m*n + n*n) doubles): every column access of a rotation is
// then an LDS access instead of an L2 round trip, which is what bounds the
// latency-bound sweeps for the small matrices of the TT splits and roundings.
// With wantv == 0 only A is resident (m*n doubles) and V is not formed.
__global__ __launch_bounds__(DT) void jacobi_svd_lds_kernel(const double* Ag, int m, int n, double* U,
                                                            double* sigma, double* V, int* order, int max_sweeps,
                                                            double tol, int* sweeps_out, int wantv) {
  extern __shared__ double lds[];
  __shared__ int s_rot[2];
  double* As = lds;
  double* Vs = wantv ? lds + (long)m * n : nullptr;
  for (long t = threadIdx.x; t < (long)m * n; t += blockDim.x) As[t] = Ag[t];
  jacobi_svd_body(As, m, n, Vs, U, sigma, V, order, max_sweeps, tol, sweeps_out, s_rot);
}

// Only A in LDS, the rotation accumulator in global memory (Vw, n*n doubles):
// for matrices whose columns fit but whose V does not (e.g. 128 x 96, or the
// n x n triangular factor of a QR for n up to 143).  Every dot product of a
// rotation reads LDS; only the shorter V updates go through L2.
__global__ __launch_bounds__(DT) void jacobi_svd_lds_a_kernel(const double* Ag, int m, int n, double* Vw, double* U,
                                                              double* sigma, double* V, int* order, int max_sweeps,
                                                              double tol, int* sweeps_out) {
  extern __shared__ double lds[];
  __shared__ int s_rot[2];
  double* As = lds;
  for (long t = threadIdx.x; t < (long)m * n; t += blockDim.x) As[t] = Ag[t];
  jacobi_svd_body(As, m, n, Vw, U, sigma, V, order, max_sweeps, tol, sweeps_out, s_rot);
}

// ---------------------------------------------------------------------------
// LU with partial pivoting of a row-major n x n matrix A and solve for nrhs
// right-hand sides B (row-major n x nrhs), in place: on exit B holds X.
// status[0] = 0 on success, j+1 if the pivot of column j is exactly zero.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(DT) void lu_solve_kernel(double* A, int n, double* B, int nrhs, int* status) {
  __shared__ double rv[DT / 64];
  __shared__ int ri[DT / 64];
  if (threadIdx.x == 0) status[0] = 0;
  for (int j = 0; j < n; ++j) {
    // pivot search (max |A[i][j]|, lowest index on ties)
    double best = -1.0; int bi = j;
    for (int i = j + threadIdx.x; i < n; i += blockDim.x) {
      double v = fabs(A[(long)i * n + j]);
      if (v > best) { best = v; bi = i; }
    }
    xlane::block_argmax<DT / 64>(best, bi, min(DT / 64, (n - j + 63) / 64), rv, ri);
    const int piv = bi;
    if (piv != j) {
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        double t = A[(long)j * n + c]; A[(long)j * n + c] = A[(long)piv * n + c]; A[(long)piv * n + c] = t;
      }
      for (int c = threadIdx.x; c < nrhs; c += blockDim.x) {
        double t = B[(long)j * nrhs + c]; B[(long)j * nrhs + c] = B[(long)piv * nrhs + c]; B[(long)piv * nrhs + c] = t;
      }
    }
    __syncthreads();
    const double d = A[(long)j * n + j];
    if (d == 0.0) {
      if (threadIdx.x == 0) status[0] = j + 1;
      return;
    }
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[(long)i * n + j] /= d;
    __syncthreads();
    const int rows = n - j - 1, cols = n - j - 1;
    for (long t = threadIdx.x; t < (long)rows * cols; t += blockDim.x) {
      int i = j + 1 + (int)(t / cols), c = j + 1 + (int)(t % cols);
      A[(long)i * n + c] -= A[(long)i * n + j] * A[(long)j * n + c];
    }
    for (long t = threadIdx.x; t < (long)rows * nrhs; t += blockDim.x) {
      int i = j + 1 + (int)(t / nrhs), c = (int)(t % nrhs);
      B[(long)i * nrhs + c] -= A[(long)i * n + j] * B[(long)j * nrhs + c];
    }
    __syncthreads();
  }
  // back substitution U x = y
  for (int j = n - 1; j >= 0; --j) {
    const double d = A[(long)j * n + j];
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) B[(long)j * nrhs + c] /= d;
    __syncthreads();
    for (long t = threadIdx.x; t < (long)j * nrhs; t += blockDim.x) {
      int i = (int)(t / nrhs), c = (int)(t % nrhs);
      B[(long)i * nrhs + c] -= A[(long)i * n + j] * B[(long)j * nrhs + c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Cholesky A = L L^T of a row-major symmetric n x n matrix, in place (lower
// triangle).  status[0] = j+1 if the j-th pivot is not positive.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(DT) void cholesky_kernel(double* A, int n, int* status) {
  __shared__ double s_d;
  __shared__ int s_bad;
  if (threadIdx.x == 0) { status[0] = 0; s_bad = 0; }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = A[(long)j * n + j];
      if (!(d > 0.0)) { status[0] = j + 1; s_bad = 1; }
      s_d = (d > 0.0) ? sqrt(d) : 1.0;
      A[(long)j * n + j] = s_d;
    }
    __syncthreads();
    if (s_bad) return;
    const double dj = s_d;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[(long)i * n + j] /= dj;
    __syncthreads();
    const int rows = n - j - 1;
    for (long t = threadIdx.x; t < (long)rows * rows; t += blockDim.x) {
      int i = j + 1 + (int)(t / rows), c = j + 1 + (int)(t % rows);
      if (c <= i) A[(long)i * n + c] -= A[(long)i * n + j] * A[(long)c * n + j];
    }
    __syncthreads();
  }
  for (long t = threadIdx.x; t < (long)n * n; t += blockDim.x) {
    int i = (int)(t / n), c = (int)(t % n);
    if (c > i) A[t] = 0.0;
  }
}

// Solve L X = B in place (L lower triangular row-major n x n, B row-major n x nrhs).
__global__ __launch_bounds__(DT) void trsm_lower_kernel(const double* L, int n, double* B, int nrhs) {
  for (int j = 0; j < n; ++j) {
    const double d = L[(long)j * n + j];
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) B[(long)j * nrhs + c] /= d;
    __syncthreads();
    const int rows = n - j - 1;
    for (long t = threadIdx.x; t < (long)rows * nrhs; t += blockDim.x) {
      int i = j + 1 + (int)(t / nrhs), c = (int)(t % nrhs);
      B[(long)i * nrhs + c] -= L[(long)i * n + j] * B[(long)j * nrhs + c];
    }
    __syncthreads();
  }
}

// Solve L^T X = B in place.
__global__ __launch_bounds__(DT) void trsm_lower_t_kernel(const double* L, int n, double* B, int nrhs) {
  for (int j = n - 1; j >= 0; --j) {
    const double d = L[(long)j * n + j];
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) B[(long)j * nrhs + c] /= d;
    __syncthreads();
    for (long t = threadIdx.x; t < (long)j * nrhs; t += blockDim.x) {
      int i = (int)(t / nrhs), c = (int)(t % nrhs);
      B[(long)i * nrhs + c] -= L[(long)j * n + i] * B[(long)j * nrhs + c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LDS-resident variants for matrices that fit the workgroup's LDS: the whole
// matrix is staged once (row stride n + 1, odd for even n, so that the column
// accesses of a wavefront fall in different banks), factorised there and
// written back.  Thread t works on columns t % 32 + 32 k and rows t / 32 +
// 32 k' of each trailing update.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(DT) void cholesky_lds_kernel(double* A, int n, int* status) {
  extern __shared__ double S[];
  __shared__ int s_bad;
  const int ld = n | 1;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5, nt = blockDim.x;
  for (int t = tid; t < n * n; t += nt) S[(t / n) * ld + t % n] = A[t];
  if (tid == 0) { status[0] = 0; s_bad = 0; }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = S[j * ld + j];
      if (!(d > 0.0)) { status[0] = j + 1; s_bad = 1; }
      S[j * ld + j] = (d > 0.0) ? sqrt(d) : 1.0;
    }
    __syncthreads();
    if (s_bad) return;
    if (j + 1 + tid < n) {   // only the threads that scale take the reciprocal
      const double inv = 1.0 / S[j * ld + j];
      for (int i = j + 1 + tid; i < n; i += nt) S[i * ld + j] *= inv;
    }
    __syncthreads();
    for (int i = j + 1 + ty; i < n; i += nt / 32) {
      const double a = S[i * ld + j];
      for (int c = j + 1 + tx; c <= i; c += 32) S[i * ld + c] -= a * S[c * ld + j];
    }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += nt) {
    const int i = t / n, c = t % n;
    A[t] = (c <= i) ? S[i * ld + c] : 0.0;
  }
}

// LU with partial pivoting and solve, as lu_solve_kernel, with A and B in LDS.
__global__ __launch_bounds__(DT) void lu_solve_lds_kernel(double* A, int n, double* B, int nrhs, int* status) {
  extern __shared__ double S[];
  __shared__ double rv[DT / 64];
  __shared__ int ri[DT / 64];
  const int ld = n | 1;
  double* Bs = S + (size_t)n * ld;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5, nt = blockDim.x;
  for (int t = tid; t < n * n; t += nt) S[(t / n) * ld + t % n] = A[t];
  for (int t = tid; t < n * nrhs; t += nt) Bs[t] = B[t];
  if (tid == 0) status[0] = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // pivot: the largest |entry| of column j from row j on, ties to the
    // smallest row
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < n; i += nt) {
      const double v = fabs(S[i * ld + j]);
      if (v > best) { best = v; bi = i; }
    }
    xlane::block_argmax<DT / 64>(best, bi, min(DT / 64, (n - j + 63) / 64), rv, ri);
    const int piv = bi;
    if (piv != j) {
      for (int c = tid; c < n; c += nt) {
        const double t = S[j * ld + c]; S[j * ld + c] = S[piv * ld + c]; S[piv * ld + c] = t;
      }
      for (int c = tid; c < nrhs; c += nt) {
        const double t = Bs[j * nrhs + c]; Bs[j * nrhs + c] = Bs[piv * nrhs + c]; Bs[piv * nrhs + c] = t;
      }
    }
    __syncthreads();
    const double d = S[j * ld + j];
    if (d == 0.0) {
      if (tid == 0) status[0] = j + 1;
      return;
    }
    if (j + 1 + tid < n) {   // only the threads that scale take the reciprocal
      const double inv = 1.0 / d;
      for (int i = j + 1 + tid; i < n; i += nt) S[i * ld + j] *= inv;
    }
    __syncthreads();
    for (int i = j + 1 + ty; i < n; i += nt / 32) {
      const double a = S[i * ld + j];
      for (int c = j + 1 + tx; c < n; c += 32) S[i * ld + c] -= a * S[j * ld + c];
      for (int c = tx; c < nrhs; c += 32) Bs[i * nrhs + c] -= a * Bs[j * nrhs + c];
    }
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    if (tid < nrhs) {
      const double inv = 1.0 / S[j * ld + j];
      for (int c = tid; c < nrhs; c += nt) Bs[j * nrhs + c] *= inv;
    }
    __syncthreads();
    for (int i = ty; i < j; i += nt / 32) {
      const double a = S[i * ld + j];
      for (int c = tx; c < nrhs; c += 32) Bs[i * nrhs + c] -= a * Bs[j * nrhs + c];
    }
    __syncthreads();
  }
  for (int t = tid; t < n * n; t += nt) A[t] = S[(t / n) * ld + t % n];
  for (int t = tid; t < n * nrhs; t += nt) B[t] = Bs[t];
}

// Triangular solves with L (MODE 0: L X = B; 1: L^T X = B; 2: both, L^T L X
// = B, the solve with a Cholesky factor) for a slab of right-hand sides per
// workgroup: workgroup g takes columns [g cb, g cb + cb) of B into LDS.  With
// stage_l the factor is staged into LDS as well (row stride n | 1), so the n
// dependent column steps read LDS instead of waiting on L2; otherwise L is read
// through the caches (every workgroup reads all of it).  The operation order
// per right-hand side is that of the separate forward and backward sweeps.
template <int MODE>
__global__ __launch_bounds__(DT) void trsm_slab_kernel(const double* L, int n, double* B, int nrhs, int cb,
                                                       int stage_l) {
  extern __shared__ double smem[];
  const int ld = n | 1;
  double* Ls = smem;
  double* Bs = smem + (stage_l ? (size_t)n * ld : 0);
  const int c0 = blockIdx.x * cb;
  const int w = min(cb, nrhs - c0);
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int c = tid % cb, rg = tid / cb, nrg = nt / cb;
  if (stage_l)
    for (int t = tid; t < n * n; t += nt) Ls[(t / n) * ld + t % n] = L[t];
  for (int t = tid; t < n * w; t += nt) Bs[(t / w) * cb + t % w] = B[(long)(t / w) * nrhs + c0 + t % w];
  __syncthreads();
  auto l_at = [&](int i, int j) { return stage_l ? Ls[i * ld + j] : L[(long)i * n + j]; };
  // threads beyond nrg full row groups (cb not dividing the thread count) stay idle
  const bool active = c < w && rg < nrg;
  if (MODE != 1) {
    for (int j = 0; j < n; ++j) {
      if (rg == 0 && active) Bs[j * cb + c] /= l_at(j, j);
      __syncthreads();
      if (active) {
        const double bj = Bs[j * cb + c];
        for (int i = j + 1 + rg; i < n; i += nrg) Bs[i * cb + c] -= l_at(i, j) * bj;
      }
      __syncthreads();
    }
  }
  if (MODE != 0) {
    for (int j = n - 1; j >= 0; --j) {
      if (rg == 0 && active) Bs[j * cb + c] /= l_at(j, j);
      __syncthreads();
      if (active) {
        const double bj = Bs[j * cb + c];
        for (int i = rg; i < j; i += nrg) Bs[i * cb + c] -= l_at(j, i) * bj;
      }
      __syncthreads();
    }
  }
  for (int t = tid; t < n * w; t += nt) B[(long)(t / w) * nrhs + c0 + t % w] = Bs[(t / w) * cb + t % w];
}

__global__ void symmetrize_kernel(double* A, int n) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)n * n) return;
  int i = (int)(t / n), j = (int)(t % n);
  if (j <= i) return;
  double v = 0.5 * (A[(long)i * n + j] + A[(long)j * n + i]);
  A[(long)i * n + j] = v;
  A[(long)j * n + i] = v;
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------

void dense_symmetrize(double* A, int n, hipStream_t s) {
  long total = (long)n * n;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, A, n);
  TT_HIP(hipGetLastError());
}

void dense_qr(double* A, int m, int n, int lda, double* tau, hipStream_t s) {
  hipLaunchKernelGGL(qr_kernel, dim3(1), dim3(DT), 0, s, A, m, n, lda, tau);
  TT_HIP(hipGetLastError());
}

void dense_qr_form_q(const double* A, int m, int n, int lda, const double* tau, double* Q, int k, int ldq,
                     hipStream_t s) {
  hipLaunchKernelGGL(qr_form_q_kernel, dim3(1), dim3(DT), 0, s, A, m, n, lda, tau, Q, k, ldq);
  TT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Smallest eigenpair of a symmetric p x p row-major matrix B: Lanczos with full
// (two-pass) reorthogonalisation, restarted from the Ritz vector.  The
// tridiagonal T_k is solved for its smallest eigenvalue by multisection of the
// Sturm count (every thread tests one point, so each round shrinks the
// bracket by the workgroup size) and for its eigenvector by inverse iteration
// with the positive definite shift theta - delta.  Q (global) holds the
// Lanczos basis, p x (kmax + 1).  A Lanczos breakdown (invariant subspace)
// continues with a deterministic pseudo-random vector orthogonal to the basis,
// so an eigenvector orthogonal to the start vector is not missed.
// ---------------------------------------------------------------------------
constexpr int LZ_MAX = 256;

__device__ __forceinline__ double lz_pseudo(int i, int j) {
  double x = sin(12.9898 * (i + 1) + 78.233 * (j + 1)) * 43758.5453;
  return x - floor(x) - 0.5;
}

// number of eigenvalues of the symmetric tridiagonal (a, b) below x
__device__ int lz_sturm(const double* a, const double* b, int k, double x) {
  int cnt = 0;
  double dd = 1.0;
  for (int i = 0; i < k; ++i) {
    const double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
    dd = a[i] - x - ((i > 0) ? bb / dd : 0.0);
    if (dd == 0.0) dd = -1e-300;
    if (dd < 0.0) ++cnt;
  }
  return cnt;
}

// Smallest eigenvalue theta of the Lanczos tridiagonal T_k (diagonal al,
// off-diagonal be[0..k-2]) by multisection of the Sturm count, and its unit
// eigenvector y by inverse iteration.  Called by the whole workgroup; theta is
// left in *s_theta, y in shared memory; h and lq (k entries each) are scratch.
__device__ void lz_ritz_min(const double* al, const double* be, int k, double* y, double* h, double* lq, double* s_lo,
                            double* s_hi, double* s_theta, int* s_first) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
      const double r = ((i > 0) ? fabs(be[i - 1]) : 0.0) + ((i + 1 < k) ? fabs(be[i]) : 0.0);
      lo = fmin(lo, al[i] - r);
      hi = fmax(hi, al[i] + r);
    }
    *s_lo = lo - 1e-300;
    *s_hi = hi + 1e-300;
  }
  __syncthreads();
  for (int round = 0; round < 8; ++round) {
    const double lo = *s_lo, hi = *s_hi;
    if (!(hi - lo > 1e-15 * (fabs(lo) + fabs(hi)) + 1e-300)) break;
    if (tid == 0) *s_first = nt;
    __syncthreads();
    const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(nt + 1);
    if (lz_sturm(al, be, k, x) >= 1) atomicMin(s_first, tid);
    __syncthreads();
    if (tid == 0) {
      const int f = *s_first;
      const double xf = (f < nt) ? lo + (hi - lo) * (double)(f + 1) / (double)(nt + 1) : hi;
      const double xp = (f > 0) ? lo + (hi - lo) * (double)f / (double)(nt + 1) : lo;
      *s_lo = xp;
      *s_hi = xf;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double theta = 0.5 * (*s_lo + *s_hi);
    *s_theta = theta;
    // inverse iteration on T - (theta - delta) I (positive definite)
    double tn = 0.0;
    for (int i = 0; i < k; ++i) tn = fmax(tn, fabs(al[i]) + ((i > 0) ? fabs(be[i - 1]) : 0.0) + ((i + 1 < k) ? fabs(be[i]) : 0.0));
    const double sh = theta - (1e-12 * tn + 1e-300);
    // LDL^T of the tridiagonal T - sh I (h holds D, lq the multipliers
    // be[i-1] / h[i-1]), factored once for the three passes
    double dprev = al[0] - sh;
    h[0] = dprev;
    for (int i = 1; i < k; ++i) {
      const double l = be[i - 1] / dprev;
      lq[i] = l;
      dprev = al[i] - sh - l * be[i - 1];
      if (dprev == 0.0) dprev = 1e-300;
      h[i] = dprev;
    }
    for (int i = 0; i < k; ++i) y[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
      // solve (T - sh I) y_new = y in place
      for (int i = 1; i < k; ++i) y[i] -= lq[i] * y[i - 1];
      for (int i = 0; i < k; ++i) y[i] /= h[i];
      for (int i = k - 2; i >= 0; --i) y[i] -= lq[i + 1] * y[i + 1];
      double nn = 0.0;
      for (int i = 0; i < k; ++i) nn += y[i] * y[i];
      nn = sqrt(nn) + 1e-300;
      for (int i = 0; i < k; ++i) y[i] /= nn;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(DT) void lanczos_min_kernel(const double* B, int p, int kmax, int restarts, double tol,
                                                         double* Q, double* v, double* lam_out, int v_init) {
  __shared__ double al[LZ_MAX], be[LZ_MAX], y[LZ_MAX], h[LZ_MAX], lq[LZ_MAX];
  __shared__ double red[NW];
  __shared__ double s_theta, s_lo, s_hi, s_bnorm;
  __shared__ int s_first;
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64, nt = blockDim.x, nw = nt / 64;
  // start vector: the caller's (a warm start) unless it is absent or zero
  if (v_init) {
    double part = 0.0;
    for (int i = tid; i < p; i += nt) part += v[i] * v[i];
    const double nv = block_sum(part, red, p);
    v_init = (nv > 0.0 && nv < 1e300) ? 1 : 0;
  }
  if (!v_init)
    for (int i = tid; i < p; i += nt) v[i] = 1.0 + 0.25 * lz_pseudo(i, 0);
  __syncthreads();
  // Frobenius norm of B (scale for tolerances)
  {
    double part = 0.0;
    for (long t = tid; t < (long)p * p; t += nt) part += B[t] * B[t];
    const double f = block_sum(part, red);
    if (tid == 0) s_bnorm = sqrt(f) + 1e-300;
  }
  __syncthreads();
  double theta = 0.0;
  for (int rs = 0; rs <= restarts; ++rs) {
    // q_0 = v / |v|
    double part = 0.0;
    for (int i = tid; i < p; i += nt) part += v[i] * v[i];
    const double nv = sqrt(block_sum(part, red, p));
    for (int i = tid; i < p; i += nt) Q[i] = v[i] / nv;
    __syncthreads();
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
      double* qj = Q + (long)j * p;
      double* wv = Q + (long)(j + 1) * p;
      // w = B q_j, one wave per row
      for (int i = w; i < p; i += nw) {
        const double* row = B + (long)i * p;
        double acc = 0.0;
        for (int c = lane; c < p; c += 64) acc += row[c] * qj[c];
        acc = wave_sum(acc);
        if (lane == 0) wv[i] = acc;
      }
      __syncthreads();
      // two passes of classical Gram-Schmidt against q_0 .. q_j
      for (int pass = 0; pass < 2; ++pass) {
        for (int t = w; t <= j; t += nw) {
          const double* qt = Q + (long)t * p;
          double acc = 0.0;
          for (int i = lane; i < p; i += 64) acc += qt[i] * wv[i];
          acc = wave_sum(acc);
          if (lane == 0) h[t] = acc;
        }
        __syncthreads();
        if (pass == 0 && tid == 0) al[j] = h[j];
        for (int i = tid; i < p; i += nt) {
          double acc = wv[i];
          for (int t = 0; t <= j; ++t) acc -= Q[(long)t * p + i] * h[t];
          wv[i] = acc;
        }
        __syncthreads();
      }
      part = 0.0;
      for (int i = tid; i < p; i += nt) part += wv[i] * wv[i];
      double bj = sqrt(block_sum(part, red, p));
      k = j + 1;
      if (k >= p) { if (tid == 0) be[j] = 0.0; __syncthreads(); break; }
      if (bj <= 1e-13 * s_bnorm) {
        // invariant subspace: continue with a pseudo-random vector orthogonal to the basis
        for (int i = tid; i < p; i += nt) wv[i] = lz_pseudo(i, j + 1 + 7919 * rs);
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
          for (int t = w; t <= j; t += nw) {
            const double* qt = Q + (long)t * p;
            double acc = 0.0;
            for (int i = lane; i < p; i += 64) acc += qt[i] * wv[i];
            acc = wave_sum(acc);
            if (lane == 0) h[t] = acc;
          }
          __syncthreads();
          for (int i = tid; i < p; i += nt) {
            double acc = wv[i];
            for (int t = 0; t <= j; ++t) acc -= Q[(long)t * p + i] * h[t];
            wv[i] = acc;
          }
          __syncthreads();
        }
        part = 0.0;
        for (int i = tid; i < p; i += nt) part += wv[i] * wv[i];
        const double nr = sqrt(block_sum(part, red, p));
        for (int i = tid; i < p; i += nt) wv[i] /= nr;
        if (tid == 0) be[j] = 0.0;
      } else {
        for (int i = tid; i < p; i += nt) wv[i] /= bj;
        if (tid == 0) be[j] = bj;
      }
      __syncthreads();
      // after 4 and 8 steps, then every 8: stop once the smallest Ritz pair of
      // T_k has converged (its residual norm is |beta_k y_k|, exact under full
      // reorthogonalisation); a warm start often converges within the first checks
      if ((k == 4 || (k >= 8 && k % 8 == 0)) && k < kmax) {
        lz_ritz_min(al, be, k, y, h, lq, &s_lo, &s_hi, &s_theta, &s_first);
        if (be[k - 1] != 0.0 && fabs(be[k - 1] * y[k - 1]) <= 0.5 * tol * s_bnorm) break;
      }
    }
    lz_ritz_min(al, be, k, y, h, lq, &s_lo, &s_hi, &s_theta, &s_first);
    __syncthreads();
    theta = s_theta;
    // Ritz vector v = Q_k y and its residual |B v - theta v|
    for (int i = tid; i < p; i += nt) {
      double acc = 0.0;
      for (int t = 0; t < k; ++t) acc += Q[(long)t * p + i] * y[t];
      v[i] = acc;
    }
    __syncthreads();
    part = 0.0;
    for (int i = w; i < p; i += nw) {
      const double* row = B + (long)i * p;
      double acc = 0.0;
      for (int c = lane; c < p; c += 64) acc += row[c] * v[c];
      acc = wave_sum(acc);
      if (lane == 0) {
        const double r = acc - theta * v[i];
        part += r * r;
      }
    }
    const double res = sqrt(block_sum(part, red));   // partials in lane 0 of every wavefront
    if (res <= tol * s_bnorm || k >= p) break;
  }
  if (tid == 0) lam_out[0] = theta;
}

// Dynamic LDS available to the Jacobi kernel: the device's per-workgroup limit
// (queried once) minus the kernel's static shared memory, opted in with
// hipFuncSetAttribute when above the 64 KiB default.
static size_t jacobi_lds_limit() {
  static size_t limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
      (void)hipGetLastError();
      return (size_t)0;
    }
    size_t lim = (size_t)v - 256;
    if (lim > 65536 - 256 &&
        (hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_lds_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess ||
         hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_svd_lds_a_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess)) {
      (void)hipGetLastError();
      lim = 65536 - 256;
    }
    return lim;
  }();
  return limit;
}

bool dense_svd_fits_lds(int m, int n) {
  return sizeof(double) * ((size_t)m * n + (size_t)n * n) <= jacobi_lds_limit();
}

void dense_svd(double* A, int m, int n, double* U, double* sigma, double* V, double* work, int* iwork,
               hipStream_t s, int max_sweeps, double tol_in) {
  // A pair counts as orthogonal below max(tol, 4 eps sqrt(m)) relative: the
  // computed inner product of two exactly orthogonal columns of length m is
  // rounding noise of about eps sqrt(m), so a tighter threshold cannot be
  // certified by the computed products.
  if (n > 4 * DT) throw Error(TT_ERR_ARG, "dense_svd: more than 4096 columns");
  const double tol = std::max(tol_in, 4.0 * 2.220446049250313e-16 * std::sqrt((double)m));
  const double bytes = 8.0 * ((double)m * n * 2 + (double)n * n + n);
  const size_t lds_bytes = sizeof(double) * ((size_t)m * n + (size_t)n * n);
  const size_t lds_a_bytes = sizeof(double) * (size_t)m * n;
  if (lds_bytes <= jacobi_lds_limit()) {
    launch_prof(PK_JACOBI_SVD, 0.0, bytes, jacobi_svd_lds_kernel, dim3(1), dim3(DT),
                (unsigned)lds_bytes, s, (const double*)A, m, n, U, sigma, V, iwork, max_sweeps, tol, iwork + n, 1);
  } else if (lds_a_bytes <= jacobi_lds_limit()) {
    launch_prof(PK_JACOBI_SVD, 0.0, bytes, jacobi_svd_lds_a_kernel, dim3(1), dim3(DT), (unsigned)lds_a_bytes, s,
                (const double*)A, m, n, work, U, sigma, V, iwork, max_sweeps, tol, iwork + n);
  } else {
    launch_prof(PK_JACOBI_SVD, 0.0, bytes, jacobi_svd_kernel, dim3(1), dim3(DT), 0u, s, A, m, n, work, U, sigma, V,
                iwork, max_sweeps, tol, iwork + n);
  }
  TT_HIP(hipGetLastError());
}

bool dense_svd_left_fits_lds(int m, int n) {
  return sizeof(double) * (size_t)m * n <= jacobi_lds_limit();
}

void dense_svd_left(double* A, int m, int n, double* U, double* sigma, int* iwork, hipStream_t s, int max_sweeps,
                    double tol_in) {
  if (n > 4 * DT) throw Error(TT_ERR_ARG, "dense_svd_left: more than 4096 columns");
  const double tol = std::max(tol_in, 4.0 * 2.220446049250313e-16 * std::sqrt((double)m));
  const double bytes = 8.0 * ((double)m * n * 2 + n);
  const size_t lds_bytes = sizeof(double) * (size_t)m * n;
  if (lds_bytes <= jacobi_lds_limit())
    launch_prof(PK_JACOBI_SVD, 0.0, bytes, jacobi_svd_lds_kernel, dim3(1), dim3(DT),
                (unsigned)lds_bytes, s, (const double*)A, m, n, U, sigma, (double*)nullptr, iwork, max_sweeps, tol,
                iwork + n, 0);
  else
    launch_prof(PK_JACOBI_SVD, 0.0, bytes, jacobi_svd_kernel, dim3(1), dim3(DT), 0u, s, A, m, n, (double*)nullptr, U,
                sigma, (double*)nullptr, iwork, max_sweeps, tol, iwork + n);
  TT_HIP(hipGetLastError());
}

void dense_sym_min_eig(const double* B, int p, double* v, double* lam, double* work, hipStream_t s, int kmax,
                       int restarts, double tol, bool v_init) {
  kmax = std::max(1, std::min({kmax, p, LZ_MAX - 1}));
  // algorithmic traffic: B read once (the iteration count is decided on the device)
  launch_prof(PK_LANCZOS, 0.0, 8.0 * (double)p * p, lanczos_min_kernel, dim3(1), dim3(DT), 0u, s, B, p, kmax,
              restarts, tol, work, v, lam, v_init ? 1 : 0);
  TT_HIP(hipGetLastError());
}

// The single-workgroup factorisations below are timed as one group; their
// algorithmic flops are the textbook counts.
// Dynamic LDS opt-in for the small dense kernels (the same device limit as the
// Jacobi kernels).
static size_t small_lds_limit() {
  static size_t limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
      (void)hipGetLastError();
      return (size_t)0;
    }
    // static shared memory of lu_solve_lds_kernel (rv, ri) is 12 KiB
    size_t lim = (size_t)v - (size_t)DT * 12 - 256;
    const void* ks[] = {reinterpret_cast<const void*>(&cholesky_lds_kernel),
                        reinterpret_cast<const void*>(&lu_solve_lds_kernel),
                        reinterpret_cast<const void*>(&trsm_slab_kernel<0>),
                        reinterpret_cast<const void*>(&trsm_slab_kernel<1>),
                        reinterpret_cast<const void*>(&trsm_slab_kernel<2>)};
    if (lim > 65536 - (size_t)DT * 12 - 256)
      for (const void* k : ks)
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess) {
          (void)hipGetLastError();
          lim = 65536 - (size_t)DT * 12 - 256;
          break;
        }
    return lim;
  }();
  return limit;
}

bool dense_small_fits_lds(int n, int nrhs) {
  return sizeof(double) * ((size_t)n * (n | 1) + (size_t)n * nrhs) <= small_lds_limit();
}

// The single-workgroup factorisations below are timed as one group; their
// algorithmic flops are the textbook counts.
void dense_lu_solve(double* A, int n, double* B, int nrhs, int* status, hipStream_t s) {
  const double nn = n;
  const double fl = 2.0 / 3.0 * nn * nn * nn + 2.0 * nn * nn * nrhs, by = 8.0 * (2.0 * nn * nn + 2.0 * nn * nrhs);
  const size_t lds = sizeof(double) * ((size_t)n * (n | 1) + (size_t)n * nrhs);
  if (lds <= small_lds_limit())
    launch_prof(PK_DENSE_1WG, fl, by, lu_solve_lds_kernel, dim3(1), dim3(DT), (unsigned)lds, s, A, n, B, nrhs, status);
  else
    launch_prof(PK_DENSE_1WG, fl, by, lu_solve_kernel, dim3(1), dim3(DT), 0u, s, A, n, B, nrhs, status);
  TT_HIP(hipGetLastError());
}

void dense_cholesky(double* A, int n, int* status, hipStream_t s) {
  const double nn = n;
  const size_t lds = sizeof(double) * (size_t)n * (n | 1);
  if (lds <= small_lds_limit())
    launch_prof(PK_DENSE_1WG, nn * nn * nn / 3.0, 8.0 * 2.0 * nn * nn, cholesky_lds_kernel, dim3(1), dim3(DT),
                (unsigned)lds, s, A, n, status);
  else
    launch_prof(PK_DENSE_1WG, nn * nn * nn / 3.0, 8.0 * 2.0 * nn * nn, cholesky_kernel, dim3(1), dim3(DT), 0u, s, A,
                n, status);
  TT_HIP(hipGetLastError());
}

// mode 0: L X = B, 1: L^T X = B, 2: L^T L X = B
static void trsm_modes(const double* L, int n, double* B, int nrhs, int mode, hipStream_t s) {
  const double nn = n;
  const double fl = (mode == 2 ? 2.0 : 1.0) * nn * nn * nrhs, by = 8.0 * (0.5 * nn * nn + 2.0 * nn * nrhs);
  // slabs of up to 16 right-hand sides, one workgroup each; the factor is
  // staged into LDS with them when both fit
  const int cb = std::min(16, std::max(1, nrhs));
  const size_t lds_b = sizeof(double) * (size_t)n * cb;
  const size_t lds_l = sizeof(double) * (size_t)n * (n | 1);
  if (lds_b <= small_lds_limit()) {
    const int stage = (lds_b + lds_l <= small_lds_limit()) ? 1 : 0;
    const unsigned lds = (unsigned)(lds_b + (stage ? lds_l : 0));
    const dim3 grid((nrhs + cb - 1) / cb);
    // about two threads per row of each right-hand side of the slab
    const dim3 blk(std::max(64, std::min(DT, ((2 * n * cb + 63) / 64) * 64)));
    if (mode == 0)
      launch_prof(PK_DENSE_1WG, fl, by, trsm_slab_kernel<0>, grid, blk, lds, s, L, n, B, nrhs, cb, stage);
    else if (mode == 1)
      launch_prof(PK_DENSE_1WG, fl, by, trsm_slab_kernel<1>, grid, blk, lds, s, L, n, B, nrhs, cb, stage);
    else
      launch_prof(PK_DENSE_1WG, fl, by, trsm_slab_kernel<2>, grid, blk, lds, s, L, n, B, nrhs, cb, stage);
  } else {
    if (mode != 1) launch_prof(PK_DENSE_1WG, fl, by, trsm_lower_kernel, dim3(1), dim3(DT), 0u, s, L, n, B, nrhs);
    if (mode != 0) launch_prof(PK_DENSE_1WG, fl, by, trsm_lower_t_kernel, dim3(1), dim3(DT), 0u, s, L, n, B, nrhs);
  }
  TT_HIP(hipGetLastError());
}

void dense_trsm_lower(const double* L, int n, double* B, int nrhs, bool transpose, hipStream_t s) {
  trsm_modes(L, n, B, nrhs, transpose ? 1 : 0, s);
}

void dense_chol_solve(const double* L, int n, double* B, int nrhs, hipStream_t s) {
  trsm_modes(L, n, B, nrhs, 2, s);
}

}  // namespace ttipm
