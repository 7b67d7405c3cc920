// Memory-bound helper kernels of the TT library: index permutations, block
// placement (TT sums by core concatenation), per-core Kronecker products and
// diag_TT cores, vector updates and deterministic dot products.
//
// These are HBM/L2-bound: each thread handles consecutive output elements so
// stores coalesce, and the reductions use a fixed two-level order (per-block
// partials, then one block) so that repeated runs are bit-identical.
#include "ttops.hpp"
#include "xlane.hpp"

namespace ttipm {

constexpr int TB = 256;

// ---------------------------------------------------------------------------
// general permutation of a dense tensor with up to 6 indices
// out[idx permuted] = alpha * in[idx] (+ beta * out)
// ---------------------------------------------------------------------------
struct PermArgs {
  int nd;
  long total;
  long in_dims[6];
  long out_stride_for_in[6];   // stride in `out` of each input index
};

__global__ void permute_kernel(const double* in, double* out, PermArgs a, double alpha) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.total) return;
  long off = 0;
  if (a.total < 2147483648L) {   // 32-bit index decomposition (see permute_many_kernel)
    unsigned rem = (unsigned)t;
    for (int i = a.nd - 1; i >= 0; --i) {
      const unsigned di = (unsigned)a.in_dims[i];
      const unsigned v = rem % di;
      rem /= di;
      off += (long)v * a.out_stride_for_in[i];
    }
  } else {
    long rem = t;
    for (int i = a.nd - 1; i >= 0; --i) {
      long v = rem % a.in_dims[i];
      rem /= a.in_dims[i];
      off += v * a.out_stride_for_in[i];
    }
  }
  out[off] = alpha * in[t];
}

void permute(const double* in, double* out, const std::vector<long>& dims, const std::vector<int>& perm,
             hipStream_t s, double alpha) {
  // out has dims[perm[0]], dims[perm[1]], ... (row-major)
  const int nd = (int)dims.size();
  TT_REQUIRE(nd >= 1 && nd <= 6 && (int)perm.size() == nd, "permute rank");
  PermArgs a;
  a.nd = nd;
  a.total = 1;
  for (int i = 0; i < nd; ++i) { a.in_dims[i] = dims[i]; a.total *= dims[i]; }
  long ostr[6];
  long st = 1;
  for (int j = nd - 1; j >= 0; --j) { ostr[j] = st; st *= dims[perm[j]]; }
  for (int j = 0; j < nd; ++j) a.out_stride_for_in[perm[j]] = ostr[j];
  if (a.total == 0) return;
  hipLaunchKernelGGL(permute_kernel, dim3(nblocks(a.total, TB)), dim3(TB), 0, s, in, out, a, alpha);
  TT_HIP(hipGetLastError());
}

// Several independent permutations in one launch: problem i owns the
// threads [end[i-1], end[i]) of a 1-D grid, one per input element.
constexpr int kPermMany = 16;
struct PermProb {
  const double* in;
  double* out;
  int nd;
  int dims[6];
  long ostr[6];
};
struct PermManyArgs {
  PermProb p[kPermMany];
  long end[kPermMany];
  int n;
};

// Index arithmetic in 32 bits (every problem holds fewer than 2^31 elements):
// the 64-bit divisions of a generic index decomposition cost more than the
// element's load and store.
__global__ void permute_many_kernel(PermManyArgs a) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.end[a.n - 1]) return;
  int i = 0;
  while (i + 1 < a.n && t >= a.end[i]) ++i;
  const PermProb& q = a.p[i];
  const unsigned local = (unsigned)(t - (i ? a.end[i - 1] : 0));
  unsigned rem = local;
  long off = 0;
  for (int j = q.nd - 1; j >= 0; --j) {
    const unsigned dj = (unsigned)q.dims[j];
    const unsigned v = rem % dj;
    rem /= dj;
    off += (long)v * q.ostr[j];
  }
  q.out[off] = q.in[local];
}

void permute_many(const std::vector<PermJob>& jobs, hipStream_t s) {
  PermManyArgs a{};
  auto flush = [&]() {
    if (a.n == 0) return;
    hipLaunchKernelGGL(permute_many_kernel, dim3(nblocks(a.end[a.n - 1], TB)), dim3(TB), 0, s, a);
    TT_HIP(hipGetLastError());
    a = PermManyArgs{};
  };
  for (const PermJob& j : jobs) {
    const int nd = (int)j.dims.size();
    TT_REQUIRE(nd >= 1 && nd <= 6 && (int)j.perm.size() == nd, "permute rank");
    PermProb& q = a.p[a.n];
    q.in = j.in;
    q.out = j.out;
    q.nd = nd;
    long total = 1;
    for (int i = 0; i < nd; ++i) {
      TT_REQUIRE(j.dims[i] >= 0 && j.dims[i] <= 2147483647L, "permute dimension");
      q.dims[i] = (int)j.dims[i];
      total *= j.dims[i];
    }
    if (total == 0) continue;
    TT_REQUIRE(total < 2147483648L, "permute_many: more than 2^31 elements in one problem");
    long st = 1;
    for (int k = nd - 1; k >= 0; --k) {
      q.ostr[j.perm[k]] = st;
      st *= j.dims[j.perm[k]];
    }
    a.end[a.n] = (a.n ? a.end[a.n - 1] : 0) + total;
    ++a.n;
    if (a.n == kPermMany) flush();
  }
  flush();
}

// ---------------------------------------------------------------------------
// dst[(o0 + i) * dst_s0 + mid * ... ] : place a [n0][mid][n1] block into a
// [N0][mid][N1] tensor at offsets (o0, o1), scaled by alpha.
// ---------------------------------------------------------------------------
__global__ void place_kernel(const double* src, int n0, long mid, int n1, double* dst, int N0, int N1, int o0,
                             int o1, double alpha) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)n0 * mid * n1;
  if (t >= total) return;
  int c = (int)(t % n1);
  long r = t / n1;
  long m = r % mid;
  int a = (int)(r / mid);
  dst[((long)(o0 + a) * mid + m) * N1 + (o1 + c)] = alpha * src[t];
}

void place_block(const double* src, int n0, long mid, int n1, double* dst, int N0, int N1, int o0, int o1,
                 double alpha, hipStream_t s) {
  long total = (long)n0 * mid * n1;
  if (total == 0) return;
  hipLaunchKernelGGL(place_kernel, dim3(nblocks(total, TB)), dim3(TB), 0, s, src, n0, mid, n1, dst, N0, N1, o0,
                     o1, alpha);
  TT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// per-core Kronecker product of two TT-matrix cores (Def. "Kronecker product
// of TT matrices"): C[(a,b)][(i,k)][(j,l)][(c,e)] = A[a][i][j][c] B[b][k][l][e]
// ---------------------------------------------------------------------------
__global__ void kron_core_kernel(const double* A, int ra, int ma, int na, int sa, const double* B, int rb, int mb,
                                 int nb, int sb, double* C) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)ra * rb * ma * mb * na * nb * sa * sb;
  if (t >= total) return;
  long r = t;
  int e = (int)(r % sb); r /= sb;
  int c = (int)(r % sa); r /= sa;
  int l = (int)(r % nb); r /= nb;
  int j = (int)(r % na); r /= na;
  int k = (int)(r % mb); r /= mb;
  int i = (int)(r % ma); r /= ma;
  int b = (int)(r % rb); r /= rb;
  int a = (int)r;
  C[t] = A[(((long)a * ma + i) * na + j) * sa + c] * B[(((long)b * mb + k) * nb + l) * sb + e];
}

void kron_core(const double* A, int ra, int ma, int na, int sa, const double* B, int rb, int mb, int nb, int sb,
               double* C, hipStream_t s) {
  long total = (long)ra * rb * ma * mb * na * nb * sa * sb;
  hipLaunchKernelGGL(kron_core_kernel, dim3(nblocks(total, TB)), dim3(TB), 0, s, A, ra, ma, na, sa, B, rb, mb,
                     nb, sb, C);
  TT_HIP(hipGetLastError());
}

// diag_TT core: D[a][i][j][b] = (i == j) v[a][i][b]
__global__ void diag_core_kernel(const double* v, int r, int m, int s, double* D) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)r * m * m * s;
  if (t >= total) return;
  long q = t;
  int b = (int)(q % s); q /= s;
  int j = (int)(q % m); q /= m;
  int i = (int)(q % m); q /= m;
  int a = (int)q;
  D[t] = (i == j) ? v[((long)a * m + i) * s + b] : 0.0;
}

void diag_core(const double* v, int r, int m, int s, double* D, hipStream_t st) {
  long total = (long)r * m * m * s;
  hipLaunchKernelGGL(diag_core_kernel, dim3(nblocks(total, TB)), dim3(TB), 0, st, v, r, m, s, D);
  TT_HIP(hipGetLastError());
}

// TT matrix-vector core: y[(a,c)][i][(b,e)] = sum_j A[a][i][j][b] x[c][j][e]
__global__ void matvec_core_kernel(const double* A, int R, int mo, int mi, int S, const double* x, int r, int s,
                                   double* y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)R * r * mo * S * s;
  if (t >= total) return;
  long q = t;
  int e = (int)(q % s); q /= s;
  int b = (int)(q % S); q /= S;
  int i = (int)(q % mo); q /= mo;
  int c = (int)(q % r); q /= r;
  int a = (int)q;
  double acc = 0.0;
  for (int j = 0; j < mi; ++j) acc += A[(((long)a * mo + i) * mi + j) * S + b] * x[((long)c * mi + j) * s + e];
  y[t] = acc;
}

void matvec_core(const double* A, int R, int mo, int mi, int S, const double* x, int r, int s, double* y,
                 hipStream_t st) {
  long total = (long)R * r * mo * S * s;
  hipLaunchKernelGGL(matvec_core_kernel, dim3(nblocks(total, TB)), dim3(TB), 0, st, A, R, mo, mi, S, x, r, s, y);
  TT_HIP(hipGetLastError());
}

// TT matrix-matrix core: C[(a,c)][i][k][(b,e)] = sum_j A[a][i][j][b] B[c][j][k][e]
__global__ void matmat_core_kernel(const double* A, int R, int mo, int mi, int S, const double* B, int r, int nk,
                                   int s, double* C) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)R * r * mo * nk * S * s;
  if (t >= total) return;
  long q = t;
  int e = (int)(q % s); q /= s;
  int b = (int)(q % S); q /= S;
  int k = (int)(q % nk); q /= nk;
  int i = (int)(q % mo); q /= mo;
  int c = (int)(q % r); q /= r;
  int a = (int)q;
  double acc = 0.0;
  for (int j = 0; j < mi; ++j)
    acc += A[(((long)a * mo + i) * mi + j) * S + b] * B[(((long)c * mi + j) * nk + k) * s + e];
  C[t] = acc;
}

void matmat_core(const double* A, int R, int mo, int mi, int S, const double* B, int r, int nk, int s, double* C,
                 hipStream_t st) {
  long total = (long)R * r * mo * nk * S * s;
  hipLaunchKernelGGL(matmat_core_kernel, dim3(nblocks(total, TB)), dim3(TB), 0, st, A, R, mo, mi, S, B, r, nk, s,
                     C);
  TT_HIP(hipGetLastError());
}

// dst[i][j] = src[i][j] for a rows x cols block with leading dimensions src_ld, dst_ld
__global__ void copy2d_kernel(const double* src, long src_ld, double* dst, long dst_ld, int rows, int cols) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)rows * cols) return;
  int i = (int)(t / cols), j = (int)(t % cols);
  dst[i * dst_ld + j] = src[i * src_ld + j];
}
void copy2d(const double* src, long src_ld, double* dst, long dst_ld, int rows, int cols, hipStream_t s) {
  long total = (long)rows * cols;
  if (total <= 0) return;
  hipLaunchKernelGGL(copy2d_kernel, dim3(nblocks(total, TB)), dim3(TB), 0, s, src, src_ld, dst, dst_ld, rows, cols);
  TT_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// vector updates
// ---------------------------------------------------------------------------
__global__ void axpby_kernel(long n, double a, const double* x, double b, double* y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = (b == 0.0 ? 0.0 : b * y[t]) + a * x[t];
}
void axpby(long n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n, TB)), dim3(TB), 0, s, n, a, x, b, y);
  TT_HIP(hipGetLastError());
}

__global__ void fill_kernel(long n, double v, double* y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = v;
}
void fill(long n, double v, double* y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n, TB)), dim3(TB), 0, s, n, v, y);
  TT_HIP(hipGetLastError());
}

// y[i] += sum_j coef[j] * V[j][i]  (V: k vectors of length n, row stride ld);  coef on device
__global__ void gemv_t_kernel(long n, int k, const double* V, long ld, const double* coef, double sign, double* y) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  // four columns at a time: their loads are in flight together, and the sum
  // keeps the order of one column at a time
  double acc = 0.0;
  for (int j0 = 0; j0 < k; j0 += 4) {
    double cs[4], vs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u;
      cs[u] = j < k ? coef[j] : 0.0;
      vs[u] = j < k ? V[(long)j * ld + t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (j0 + u < k) acc += cs[u] * vs[u];
  }
  y[t] += sign * acc;
}
void gemv_update(long n, int k, const double* V, long ld, const double* coef, double sign, double* y,
                 hipStream_t s) {
  if (n <= 0 || k <= 0) return;
  hipLaunchKernelGGL(gemv_t_kernel, dim3(nblocks(n, TB)), dim3(TB), 0, s, n, k, V, ld, coef, sign, y);
  TT_HIP(hipGetLastError());
}

// Deterministic multi-dot: out[j] = <V_j, w> for k vectors.  Short vectors
// take one workgroup per product; longer ones a two-stage reduction (stage 1
// writes per-block partials part[j][blk], stage 2 sums them in index order).
constexpr int DOT_BLOCKS = 256;

__global__ void mdot_stage1(long n, int k, const double* V, long ld, const double* w, double* part) {
  __shared__ double red[TB / 64];
  const int j = blockIdx.y;
  const double* v = V + (long)j * ld;
  double acc = 0.0;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    acc += v[t] * w[t];
  acc = xlane::wave_sum(acc);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < TB / 64; ++i) s += red[i];
    part[(long)j * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void mdot_stage2(int nb, int k, const double* part, double* out) {
  const int j = blockIdx.x;
  __shared__ double red[TB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[(long)j * nb + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

// Vectors up to this length: one workgroup per dot product, one launch.
constexpr long DOT_SINGLE_MAX = 32768;

__global__ void mdot_single(long n, const double* V, long ld, const double* w, double* out) {
  __shared__ double red[TB / 64];
  const int j = blockIdx.x;
  const double* v = V + (long)j * ld;
  double acc = 0.0;
  // four entries per thread at a time: the loads are issued before the first
  // product waits on them, and the sum keeps the order of one entry at a time
  constexpr int U = 4;
  for (long t0 = threadIdx.x; t0 < n; t0 += (long)U * blockDim.x) {
    double vs[U], ws[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long t = t0 + (long)u * blockDim.x;
      vs[u] = t < n ? v[t] : 0.0;
      ws[u] = t < n ? w[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (t0 + (long)u * blockDim.x < n) acc += vs[u] * ws[u];
  }
  acc = xlane::wave_sum(acc);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int i = 0; i < TB / 64; ++i) sum += red[i];
    out[j] = sum;
  }
}

void mdot(long n, int k, const double* V, long ld, const double* w, double* out, double* part, hipStream_t s) {
  if (k <= 0) return;
  if (n <= DOT_SINGLE_MAX) {
    hipLaunchKernelGGL(mdot_single, dim3(k), dim3(TB), 0, s, n, V, ld, w, out);
    TT_HIP(hipGetLastError());
    return;
  }
  int nb = (int)std::min<long>(DOT_BLOCKS, std::max<long>(1, (n + TB - 1) / TB));
  hipLaunchKernelGGL(mdot_stage1, dim3(nb, k), dim3(TB), 0, s, n, k, V, ld, w, part);
  TT_HIP(hipGetLastError());
  hipLaunchKernelGGL(mdot_stage2, dim3(k), dim3(TB), 0, s, nb, k, part, out);
  TT_HIP(hipGetLastError());
}

size_t mdot_part_size(int k) { return (size_t)k * DOT_BLOCKS; }

}  // namespace ttipm
