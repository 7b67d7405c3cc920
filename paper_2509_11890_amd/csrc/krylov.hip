// Restarted GMRES (classical Gram-Schmidt applied twice) with right
// preconditioning and a mixed-precision refinement mode, and the block-Jacobi
// preconditioner of the projected local operators (Sec. 3.3).
#include "krylov.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "ttops.hpp"

namespace ttipm {

double dev_norm(const double* x, long n, Ctx& c);

namespace {

// One Arnoldi column on the device: h[0..j] are the projections of the new
// vector and h[j+1] its squared norm after orthogonalisation.  Stores the
// column into H (row-major, (m+1) x m), applies the previous Givens rotations,
// forms rotation j, updates the rotated right-hand side g, and records the
// residual estimate |g[j+1]|, the norm hn and the scale 1/hn of the new vector.
__global__ void arnoldi_givens_kernel(int j, int m, const double* h, double* H, double* cs, double* sn, double* g,
                                      double* res, double* hns, double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double hn = sqrt(fmax(h[j + 1], 0.0));
  for (int i = 0; i <= j; ++i) H[(long)i * m + j] = h[i];
  H[(long)(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = H[(long)i * m + j], b = H[(long)(i + 1) * m + j];
    H[(long)i * m + j] = cs[i] * a + sn[i] * b;
    H[(long)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[(long)j * m + j], b = H[(long)(j + 1) * m + j];
  const double rr = hypot(a, b);
  cs[j] = (rr == 0.0) ? 1.0 : a / rr;
  sn[j] = (rr == 0.0) ? 0.0 : b / rr;
  H[(long)j * m + j] = rr;
  H[(long)(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  res[j] = fabs(g[j + 1]);
  hns[j] = hn;
  scal[0] = (hn > 0.0) ? 1.0 / hn : 0.0;
}

// x *= scal[0] (device scalar)
__global__ void scale_dev_kernel(long n, double* x, const double* scal) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= scal[0];
}

__global__ void set_first_kernel(double* g, int len, double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) g[i] = (i == 0) ? beta : 0.0;
}

// Back substitution of the cycle's least-squares problem: y solves the upper
// triangular H[0:len, 0:len] y = g[0:len] (H row-major with row stride m), a
// zero diagonal entry giving y_i = 0.  With staged != 0 the wavefront first
// copies the len x len block into LDS (dynamic, len * len doubles); one lane
// then runs the substitution row by row, each row's sum left to right with
// separately rounded products and differences (no contraction), the
// arithmetic of the textbook loop.
__global__ __launch_bounds__(64) void backsub_kernel(const double* H, int m, const double* g, int len, double* y,
                                                     int staged) {
#pragma clang fp contract(off)
  extern __shared__ double Hs[];
  if (staged)
    for (int t = threadIdx.x; t < len * len; t += 64) Hs[t] = H[(long)(t / len) * m + t % len];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double* R = staged ? Hs : H;
  const long ld = staged ? len : m;
  for (int i = len - 1; i >= 0; --i) {
    double acc = g[i];
    for (int l = i + 1; l < len; ++l) acc -= R[i * ld + l] * y[l];
    y[i] = (R[i * ld + i] != 0.0) ? acc / R[i * ld + i] : 0.0;
  }
}

}  // namespace

// Arnoldi steps run without host round trips: the Givens rotations are applied
// on the device and the host reads the residual estimates every kCheck steps
// (and at the end of a cycle).  A cycle that converged inside such a block
// keeps only the columns up to the converged step (the rotated system of a
// prefix is final once its step is done), so the extra steps cost time only;
// info.iters counts the steps the solution uses.
void gmres_solve(long n, const KrylovOps& ops, const double* f, double* u, const KrylovParams& prm, KrylovInfo& info,
                 Ctx& c) {
  constexpr int kCheck = 4;
  const int m = std::max(1, prm.restart);
  DevBuf V((size_t)(m + 1) * n), r0(n), z(n), w(n), h(m + 2), h2(m + 2), yv(m + 1);
  DevBuf Hd((size_t)(m + 1) * m), csd(m), snd(m), gd(m + 1), resd(m), hnd(m), scal(2);
  c.dot_part.reserve(mdot_part_size(m + 1));
  info = KrylovInfo{};
  const double bn = dev_norm(f, n, c);
  if (bn == 0.0) {
    fill(n, 0.0, u, c.s);
    c.sync();
    return;
  }
  double best = std::numeric_limits<double>::infinity();
  int stall = 0;
  while (true) {
    ops.matvec(u, r0.get(), false);                 // true residual in FP64
    axpby(n, 1.0, f, -1.0, r0.get(), c.s);
    const double beta = dev_norm(r0.get(), n, c);
    info.rel_res = beta / bn;
    if (info.rel_res <= prm.rtol || info.iters >= prm.maxit) break;
    if (prm.mixed) {                                 // refinement that stops reducing the residual
      if (info.rel_res > 0.5 * best) {
        if (++stall >= 3) break;
      } else {
        stall = 0;
      }
      best = std::min(best, info.rel_res);
    }
    const double target = prm.mixed ? std::max(prm.rtol * bn, prm.inner_tol * beta) : prm.rtol * bn;
    axpby(n, 1.0 / beta, r0.get(), 0.0, V.get(), c.s);
    hipLaunchKernelGGL(set_first_kernel, dim3(nblocks(m + 1, 64)), dim3(64), 0, c.s, gd.get(), m + 1, beta);
    TT_HIP(hipGetLastError());
    int j = 0, jend = -1, jchk = 0;
    for (; j < m && info.iters < prm.maxit; ++j) {
      ++info.iters;
      const double* vj = V.get() + (size_t)j * n;
      double* v1 = V.get() + (size_t)(j + 1) * n;
      if (ops.precond) {
        ops.precond(vj, z.get());
        ops.matvec(z.get(), v1, prm.mixed);
      } else {
        ops.matvec(vj, v1, prm.mixed);
      }
      mdot(n, j + 1, V.get(), n, v1, h.get(), c.dot_part.get(), c.s);
      gemv_update(n, j + 1, V.get(), n, h.get(), -1.0, v1, c.s);
      mdot(n, j + 1, V.get(), n, v1, h2.get(), c.dot_part.get(), c.s);
      gemv_update(n, j + 1, V.get(), n, h2.get(), -1.0, v1, c.s);
      axpby(j + 1, 1.0, h2.get(), 1.0, h.get(), c.s);
      mdot(n, 1, v1, n, v1, h.get() + j + 1, c.dot_part.get(), c.s);
      hipLaunchKernelGGL(arnoldi_givens_kernel, dim3(1), dim3(64), 0, c.s, j, m, h.get(), Hd.get(), csd.get(),
                         snd.get(), gd.get(), resd.get(), hnd.get(), scal.get());
      hipLaunchKernelGGL(scale_dev_kernel, dim3(nblocks(n, 256)), dim3(256), 0, c.s, n, v1, scal.get());
      TT_HIP(hipGetLastError());
      const bool last = (j + 1 == m) || (info.iters >= prm.maxit);
      if ((j + 1 - jchk) >= kCheck || last) {
        // residual estimates and norms of steps jchk .. j
        const int cnt = j + 1 - jchk;
        double* hh = c.host(2 * m + 2);   // pinned: residual estimates and norms of the block
        TT_HIP(hipMemcpyAsync(hh, resd.get() + jchk, sizeof(double) * cnt, hipMemcpyDeviceToHost, c.s));
        TT_HIP(hipMemcpyAsync(hh + m + 1, hnd.get() + jchk, sizeof(double) * cnt, hipMemcpyDeviceToHost, c.s));
        c.sync();
        for (int t = 0; t < cnt; ++t) {
          if (hh[t] <= target || hh[m + 1 + t] == 0.0) {
            jend = jchk + t + 1;
            break;
          }
        }
        jchk = j + 1;
        if (jend >= 0) break;
      }
    }
    if (jend < 0) {
      jend = j;
    } else {
      info.iters -= (j + 1) - jend;   // steps computed past the converged one are not part of the solve
    }
    // back substitution on the device with the final rotated columns 0 .. jend-1
    if (jend > 0) {
      const size_t lds = sizeof(double) * (size_t)jend * jend;
      const int staged = lds <= 65536 ? 1 : 0;
      hipLaunchKernelGGL(backsub_kernel, dim3(1), dim3(64), staged ? (unsigned)lds : 0u, c.s, Hd.get(), m, gd.get(),
                         jend, yv.get(), staged);
      TT_HIP(hipGetLastError());
      fill(n, 0.0, z.get(), c.s);
      gemv_update(n, jend, V.get(), n, yv.get(), 1.0, z.get(), c.s);      // z = V y
      if (ops.precond) {
        ops.precond(z.get(), w.get());
        axpby(n, 1.0, w.get(), 1.0, u, c.s);
      } else {
        axpby(n, 1.0, z.get(), 1.0, u, c.s);
      }
    }
    ++info.cycles;
  }
}

// ---------------------------------------------------------------------------
// block-Jacobi preconditioner
// ---------------------------------------------------------------------------
namespace {

// out[a][alpha] = phi[a][alpha][a]
__global__ void env_diag_kernel(const double* phi, int r, int R, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * R) return;
  const int a = t / R, al = t % R;
  out[t] = phi[((long)a * R + al) * r + a];
}

// identity operator: D[a][i][j][b] = dL[a] dR[b] delta_ij
__global__ void diag_identity_kernel(const double* dL, const double* dR, int r, int m, int s, double* D) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)r * m * m * s;
  if (t >= tot) return;
  const int b = (int)(t % s);
  const int j = (int)((t / s) % m);
  const int i = (int)((t / ((long)s * m)) % m);
  const int a = (int)(t / ((long)s * m * m));
  D[t] = (i == j) ? dL[a] * dR[b] : 0.0;
}

// E[a][i][j][b] = sum_k D1[a][i][k][b] D0[a][k][j][b]
__global__ void diag_chain_kernel(const double* D1, const double* D0, int r, int m, int s, double* E) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)r * m * m * s;
  if (t >= tot) return;
  const int b = (int)(t % s);
  const int j = (int)((t / s) % m);
  const int i = (int)((t / ((long)s * m)) % m);
  const int a = (int)(t / ((long)s * m * m));
  double acc = 0.0;
  for (int k = 0; k < m; ++k)
    acc += D1[(((long)a * m + i) * m + k) * s + b] * D0[(((long)a * m + k) * m + j) * s + b];
  E[t] = acc;
}

// blk[(a,b)][row*m + i][col*m + j] += coeff D[a][i][j][b]
__global__ void diag_scatter_kernel(const double* D, int r, int m, int s, int L, int row, int col, double coeff,
                                    double* blk) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)r * m * m * s;
  if (t >= tot) return;
  const int b = (int)(t % s);
  const int j = (int)((t / s) % m);
  const int i = (int)((t / ((long)s * m)) % m);
  const int a = (int)(t / ((long)s * m * m));
  const int n = L * m;
  blk[((long)a * s + b) * n * n + (long)(row * m + i) * n + (col * m + j)] += coeff * D[t];
}

// In-place Gauss-Jordan inversion with partial pivoting, one thread per block
// (n <= 16); W is per-block scratch of n * n doubles.  Singular blocks become I.
// One thread per block, Gauss-Jordan with partial pivoting on the block and
// the identity beside it.  Both sit in LDS, entry-major and thread-minor
// (entry e of thread t at e * blockDim.x + t), so that the threads' dependent
// accesses are LDS round trips, conflict-free, instead of global ones.
__global__ void block_inverse_kernel(double* blk, int nblk, int n) {
  extern __shared__ double lds[];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblk) return;
  const int T = blockDim.x, nn = n * n;
  double* A = lds + threadIdx.x;            // entry e at A[e * T]
  double* B = lds + (long)nn * T + threadIdx.x;
  double* G = blk + (long)t * nn;
  for (int i = 0; i < nn; ++i) {
    A[i * T] = G[i];
    B[i * T] = (i / n == i % n) ? 1.0 : 0.0;
  }
  double amax = 0.0;
  for (int i = 0; i < nn; ++i) amax = fmax(amax, fabs(A[i * T]));
  bool ok = amax > 0.0;
  for (int k = 0; k < n && ok; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(A[(i * n + k) * T]) > fabs(A[(p * n + k) * T])) p = i;
    if (!(fabs(A[(p * n + k) * T]) > 1e-14 * amax)) { ok = false; break; }
    if (p != k)
      for (int j = 0; j < n; ++j) {
        double x = A[(k * n + j) * T]; A[(k * n + j) * T] = A[(p * n + j) * T]; A[(p * n + j) * T] = x;
        x = B[(k * n + j) * T]; B[(k * n + j) * T] = B[(p * n + j) * T]; B[(p * n + j) * T] = x;
      }
    const double d = 1.0 / A[(k * n + k) * T];
    for (int j = 0; j < n; ++j) { A[(k * n + j) * T] *= d; B[(k * n + j) * T] *= d; }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[(i * n + k) * T];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[(i * n + j) * T] -= f * A[(k * n + j) * T];
        B[(i * n + j) * T] -= f * B[(k * n + j) * T];
      }
    }
  }
  for (int i = 0; i < nn; ++i) G[i] = ok ? B[i * T] : ((i / n == i % n) ? 1.0 : 0.0);
}

// y[l][a][i][b] = sum_{l', j} inv[(a,b)][l m + i][l' m + j] x[l'][a][j][b]
__global__ void block_apply_kernel(const double* inv, const double* x, double* y, int r, int m, int s, int L) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long p = (long)r * m * s;
  if (t >= (long)L * p) return;
  const int b = (int)(t % s);
  const int i = (int)((t / s) % m);
  const int a = (int)((t / ((long)s * m)) % r);
  const int l = (int)(t / p);
  const int n = L * m;
  const double* M = inv + ((long)a * s + b) * n * n + (long)(l * m + i) * n;
  double acc = 0.0;
  for (int l2 = 0; l2 < L; ++l2)
    for (int j = 0; j < m; ++j) acc += M[l2 * m + j] * x[(long)l2 * p + ((long)a * m + j) * s + b];
  y[t] = acc;
}

}  // namespace

void BlockJacobi::init(int r_, int s_, int m_, int L_, Ctx& c) {
  r = r_; s = s_; m = m_; L = L_;
  const long n = (long)L * m;
  blk.reserve((size_t)r * s * n * n);
  fill((long)r * s * n * n, 0.0, blk.get(), c.s);
}

void BlockJacobi::copy_from(const BlockJacobi& o, Ctx& c) {
  r = o.r; s = o.s; m = o.m; L = o.L;
  const size_t cnt = (size_t)r * s * (L * m) * (L * m);
  blk.reserve(cnt);
  TT_HIP(hipMemcpyAsync(blk.get(), o.blk.get(), sizeof(double) * cnt, hipMemcpyDeviceToDevice, c.s));
}

void BlockJacobi::add(int row, int col, double coeff, const Op* chain, int nchain, Ctx& c) {
  const long nD = (long)r * m * m * s;
  DevBuf D[2], E(nD), dL, dR, T;
  for (int q = 0; q < nchain; ++q) {
    const Op& o = chain[q];
    D[q].reserve(nD);
    dL.reserve((size_t)r * o.R);
    dR.reserve((size_t)s * o.Rp);
    hipLaunchKernelGGL(env_diag_kernel, dim3(nblocks((size_t)r * o.R, 256)), dim3(256), 0, c.s, o.phiL, r, o.R,
                       dL.get());
    hipLaunchKernelGGL(env_diag_kernel, dim3(nblocks((size_t)s * o.Rp, 256)), dim3(256), 0, c.s, o.phiR, s, o.Rp,
                       dR.get());
    if (!o.core) {
      hipLaunchKernelGGL(diag_identity_kernel, dim3(nblocks(nD, 256)), dim3(256), 0, c.s, dL.get(), dR.get(), r, m, s,
                         D[q].get());
    } else {
      // T[a][(i,j,beta)] = sum_alpha dL[a][alpha] O[alpha][(i,j,beta)]
      T.reserve((size_t)r * m * m * o.Rp);
      gemm(gemm_nn(r, m * m * o.Rp, o.R, dL.get(), o.R, o.core, (long)m * m * o.Rp, T.get(), (long)m * m * o.Rp),
           c.s, &c.ws, GemmPrec::F64);
      // D[(a,i,j)][b] = sum_beta T[(a,i,j)][beta] dR[b][beta]
      Gemm g;
      g.M = r * m * m; g.N = s; g.K = o.Rp;
      g.A = T.get(); g.am = o.Rp; g.ak = 1;
      g.B = dR.get(); g.bk = 1; g.bn = o.Rp;
      g.C = D[q].get(); g.cm = s; g.cn = 1;
      gemm(g, c.s, &c.ws, GemmPrec::F64);
    }
    TT_HIP(hipGetLastError());
    c.sync();   // dL / dR / T are reused for the next operator of the chain
  }
  const double* Dsum = D[0].get();
  if (nchain == 2) {
    hipLaunchKernelGGL(diag_chain_kernel, dim3(nblocks(nD, 256)), dim3(256), 0, c.s, D[1].get(), D[0].get(), r, m, s,
                       E.get());
    Dsum = E.get();
  }
  hipLaunchKernelGGL(diag_scatter_kernel, dim3(nblocks(nD, 256)), dim3(256), 0, c.s, Dsum, r, m, s, L, row, col, coeff,
                     blk.get());
  TT_HIP(hipGetLastError());
  c.sync();
}

void BlockJacobi::invert(Ctx& c) {
  const int n = L * m;
  TT_REQUIRE(n <= 16, "block-Jacobi blocks are limited to 16 x 16");
  const int nb = r * s;
  // threads per workgroup: up to 64, as many as keep both n x n arrays of every
  // thread within the 64 KiB of LDS a workgroup gets without opting in
  int T = 64;
  while (T > 1 && (size_t)2 * n * n * T * sizeof(double) > 65536) T /= 2;
  TT_REQUIRE((size_t)2 * n * n * T * sizeof(double) <= 65536, "block-Jacobi block too large");
  hipLaunchKernelGGL(block_inverse_kernel, dim3(nblocks(nb, T)), dim3(T), (size_t)2 * n * n * T * sizeof(double),
                     c.s, blk.get(), nb, n);
  TT_HIP(hipGetLastError());
}

void BlockJacobi::apply(const double* x, double* y, Ctx& c) const {
  const long tot = (long)L * r * m * s;
  hipLaunchKernelGGL(block_apply_kernel, dim3(nblocks(tot, 256)), dim3(256), 0, c.s, blk.get(), x, y, r, m, s, L);
  TT_HIP(hipGetLastError());
}

}  // namespace ttipm
