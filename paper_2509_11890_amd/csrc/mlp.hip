// Learned block preconditioner: FP32 network kernels (forward, backward, Adam)
// and the block features / probe data of local systems.
#include "mlp.hpp"

#include <algorithm>
#include <cmath>
#include <random>

#include "ttops.hpp"

namespace ttipm {

double dev_norm(const double* x, long n, Ctx& c);

namespace {

// ---------------------------------------------------------------------------
// FP32 strided GEMM: C(m, n) = alpha sum_k A(m, k) B(k, n) + beta C(m, n),
// 64 x 64 tiles, 256 threads with 4 x 4 outputs each, LDS-staged k-tiles of 16.
// ---------------------------------------------------------------------------
struct SArgs {
  int M, N, K;
  const float* A; long am, ak;
  const float* B; long bk, bn;
  float* C; long cm, cn;
  float alpha, beta;
};

__global__ __launch_bounds__(256) void sgemm_kernel(SArgs g) {
  __shared__ float As[16][64 + 1];
  __shared__ float Bs[16][64 + 1];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int tm = (tid / 16) * 4, tn = (tid % 16) * 4;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int kk = e / 64, mm = e % 64;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < g.M && gk < g.K) ? g.A[gm * g.am + gk * g.ak] : 0.f;
      const int gn = n0 + mm;
      Bs[kk][mm] = (gn < g.N && gk < g.K) ? g.B[gk * g.bk + gn * g.bn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = m0 + tm + i, cc = n0 + tn + j;
      if (r < g.M && cc < g.N) {
        float* p = g.C + r * g.cm + cc * g.cn;
        *p = (g.beta == 0.f) ? g.alpha * acc[i][j] : g.alpha * acc[i][j] + g.beta * (*p);
      }
    }
}

void sgemm(int M, int N, int K, const float* A, long am, long ak, const float* B, long bk, long bn, float* C, long cm,
           long cn, float alpha, float beta, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  SArgs g{M, N, K, A, am, ak, B, bk, bn, C, cm, cn, alpha, beta};
  dim3 grid((M + 63) / 64, (N + 63) / 64);
  hipLaunchKernelGGL(sgemm_kernel, grid, dim3(256), 0, s, g);
  TT_HIP(hipGetLastError());
}

// z[j][h] += b[h]; h = relu(z)
__global__ void bias_relu_kernel(float* z, float* hout, const float* b, long N, int H) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * H) return;
  const float v = z[t] + b[t % H];
  z[t] = v;
  hout[t] = v > 0.f ? v : 0.f;
}

__global__ void bias_kernel(float* o, const float* b, long N, int O) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * O) return;
  o[t] += b[t % O];
}

// per block j: e_p = r_p - C y_p / s, loss_j = sum_p w_p |e_p|^2,
// dout_j = -(2 / N)(1 / s) sum_p w_p e_p y_p^T
__global__ void mlp_loss_kernel(const float* o, const float* R, const float* Y, const float* S, const float* W, int N,
                                int P, int n, float* loss_j, float* dout) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const float* C = o + (long)j * n * n;
  float* D = dout + (long)j * n * n;
  for (int q = 0; q < n * n; ++q) D[q] = 0.f;
  const float is = 1.f / S[j];
  const float sc = -2.f * is / (float)N;
  double lj = 0.0;
  for (int p = 0; p < P; ++p) {
    const float* r = R + ((long)j * P + p) * n;
    const float* y = Y + ((long)j * P + p) * n;
    const float w = W[(long)j * P + p];
    for (int i = 0; i < n; ++i) {
      float cy = 0.f;
      for (int k = 0; k < n; ++k) cy = fmaf(C[i * n + k], y[k], cy);
      const float e = r[i] - cy * is;
      lj += (double)w * e * e;
      for (int k = 0; k < n; ++k) D[i * n + k] += sc * w * e * y[k];
    }
  }
  loss_j[j] = (float)lj;
}

__global__ void relu_back_kernel(float* d, const float* z, long total) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < total && !(z[t] > 0.f)) d[t] = 0.f;
}

// col[c] = sum_j X[j][c] (fixed order)
__global__ void colsum_kernel(const float* X, long N, int Cn, float* col) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Cn) return;
  float s = 0.f;
  for (long j = 0; j < N; ++j) s += X[j * Cn + c];
  col[c] = s;
}

__global__ void sum_kernel(const float* x, long n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (long i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                            float c1, float c2, float eps) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// block features: F[b] = [D_b / s_b, log10 s_b, ctx], S[b] = |D_b|_F
__global__ void block_features_kernel(const double* blk, int nb, int n, const float* ctx, float* F, float* S) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double* D = blk + (long)b * n * n;
  double s = 0.0;
  for (int q = 0; q < n * n; ++q) s += D[q] * D[q];
  s = sqrt(s);
  const double is = s > 0.0 ? 1.0 / s : 0.0;
  float* f = F + (long)b * (n * n + 5);
  for (int q = 0; q < n * n; ++q) f[q] = (float)(D[q] * is);
  f[n * n] = (float)log10(s > 0.0 ? s : 1.0);
  for (int q = 0; q < 4; ++q) f[n * n + 1 + q] = ctx[q];
  S[b] = (float)(s > 0.0 ? s : 1.0);
}

// counter-based standard normals (Box-Muller on a 64-bit mix of (seed, i))
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void normal_kernel(double* x, long n, unsigned long long seed) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const unsigned long long a = mix64(seed * 0x100000001B3ull + 2 * t), b = mix64(seed * 0x100000001B3ull + 2 * t + 1);
  const double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  x[t] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// probe data of block (a,b): R = x_b - inv_b y_b, Y = y_b (float), W = w
__global__ void probe_kernel(const double* inv, const double* x, const double* y, int r, int m, int s, int L, int P,
                             int p, float w, float* R, float* Y, float* W) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = L * m;
  const long nb = (long)r * s;
  if (t >= nb * n) return;
  const long bidx = t / n;
  const int row = (int)(t % n);
  const int a = (int)(bidx / s), b = (int)(bidx % s);
  const long pp = (long)r * m * s;
  auto gidx = [&](int q) { return (long)(q / m) * pp + ((long)a * m + (q % m)) * s + b; };
  const double* M = inv + bidx * n * n + (long)row * n;
  double acc = 0.0;
  for (int q = 0; q < n; ++q) acc += M[q] * y[gidx(q)];
  R[(bidx * P + p) * n + row] = (float)(x[gidx(row)] - acc);
  Y[(bidx * P + p) * n + row] = (float)y[gidx(row)];
  if (row == 0) W[bidx * P + p] = w;
}

// rows idx[t] of src (per floats each) -> dst row t
__global__ void gather_rows_kernel(const float* src, const int* idx, long nrows, long per, float* dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows * per) return;
  const long r = t / per, q = t % per;
  dst[t] = src[(long)idx[r] * per + q];
}

__global__ void add_correction_kernel(double* inv, const float* o, const float* S, long nb, int n) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * n * n) return;
  const long b = t / ((long)n * n);
  inv[t] += (double)o[t] / (double)S[b];
}

}  // namespace

void Mlp::init(int in_, int H_, int out_, unsigned long long seed, Ctx& c) {
  in = in_; H = H_; out = out_;
  nparams = (long)H * in + H + (long)H * H + H + (long)out * H + out;
  params.reserve(nparams);
  grad.reserve(nparams);
  adam_m.reserve(nparams);
  adam_v.reserve(nparams);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<float> h(nparams, 0.f);
  float* p = h.data();
  for (long i = 0; i < (long)H * in; ++i) p[i] = (float)(nd(rng) * std::sqrt(2.0 / in));
  p += (long)H * in + H;
  for (long i = 0; i < (long)H * H; ++i) p[i] = (float)(nd(rng) * std::sqrt(2.0 / H));
  // output layer starts at zero: the network is the block-Jacobi preconditioner until trained
  TT_HIP(hipMemcpyAsync(params.get(), h.data(), sizeof(float) * nparams, hipMemcpyHostToDevice, c.s));
  TT_HIP(hipMemsetAsync(adam_m.get(), 0, sizeof(float) * nparams, c.s));
  TT_HIP(hipMemsetAsync(adam_v.get(), 0, sizeof(float) * nparams, c.s));
  adam_t = 0;
  c.sync();
}

void Mlp::forward(const float* F, int N, float* outp, Ctx& c) {
  z1.reserve((size_t)N * H); h1.reserve((size_t)N * H); z2.reserve((size_t)N * H); h2.reserve((size_t)N * H);
  sgemm(N, H, in, F, in, 1, W1(), 1, in, z1.get(), H, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(bias_relu_kernel, dim3(nblocks((size_t)N * H, 256)), dim3(256), 0, c.s, z1.get(), h1.get(), b1(),
                     (long)N, H);
  sgemm(N, H, H, h1.get(), H, 1, W2(), 1, H, z2.get(), H, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(bias_relu_kernel, dim3(nblocks((size_t)N * H, 256)), dim3(256), 0, c.s, z2.get(), h2.get(), b2(),
                     (long)N, H);
  sgemm(N, out, H, h2.get(), H, 1, W3(), 1, H, outp, out, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(bias_kernel, dim3(nblocks((size_t)N * out, 256)), dim3(256), 0, c.s, outp, b3(), (long)N, out);
  TT_HIP(hipGetLastError());
}

double Mlp::loss_grad(const MlpBatch& b, Ctx& c) {
  const int N = b.N;
  TT_REQUIRE(b.n * b.n == out, "block size does not match the network output");
  o.reserve((size_t)N * out);
  dout.reserve((size_t)N * out);
  dh.reserve((size_t)N * H);
  forward(b.F, N, o.get(), c);
  FBuf lj(N);
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(nblocks(N, 64)), dim3(64), 0, c.s, o.get(), b.R, b.Y, b.S, b.W, N, b.P,
                     b.n, lj.get(), dout.get());
  DevBuf lsum(1);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, c.s, lj.get(), (long)N, lsum.get());
  float* gW1 = grad.get();
  float* gb1 = gW1 + (long)H * in;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (long)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + (long)out * H;
  // layer 3
  sgemm(out, H, N, dout.get(), 1, out, h2.get(), H, 1, gW3, H, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(out, 64)), dim3(64), 0, c.s, dout.get(), (long)N, out, gb3);
  sgemm(N, H, out, dout.get(), out, 1, W3(), H, 1, dh.get(), H, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(relu_back_kernel, dim3(nblocks((size_t)N * H, 256)), dim3(256), 0, c.s, dh.get(), z2.get(),
                     (long)N * H);
  // layer 2 (dh holds dz2)
  sgemm(H, H, N, dh.get(), 1, H, h1.get(), H, 1, gW2, H, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(H, 64)), dim3(64), 0, c.s, dh.get(), (long)N, H, gb2);
  FBuf dh1((size_t)N * H);
  sgemm(N, H, H, dh.get(), H, 1, W2(), H, 1, dh1.get(), H, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(relu_back_kernel, dim3(nblocks((size_t)N * H, 256)), dim3(256), 0, c.s, dh1.get(), z1.get(),
                     (long)N * H);
  // layer 1
  sgemm(H, in, N, dh1.get(), 1, H, b.F, in, 1, gW1, in, 1, 1.f, 0.f, c.s);
  hipLaunchKernelGGL(colsum_kernel, dim3(nblocks(H, 64)), dim3(64), 0, c.s, dh1.get(), (long)N, H, gb1);
  TT_HIP(hipGetLastError());
  double loss = 0.0;
  TT_HIP(hipMemcpyAsync(&loss, lsum.get(), sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return loss / N;
}

void Mlp::adam_step(float lr, Ctx& c) {
  ++adam_t;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)adam_t), c2 = 1.f - std::pow(b2, (float)adam_t);
  hipLaunchKernelGGL(adam_kernel, dim3(nblocks(nparams, 256)), dim3(256), 0, c.s, params.get(), grad.get(),
                     adam_m.get(), adam_v.get(), nparams, lr, b1, b2, c1, c2, 1e-8f);
  TT_HIP(hipGetLastError());
}

void Mlp::append(const MlpBatch& b, long cap, Ctx& c) {
  if (b.N <= 0) return;
  if (ds_N == 0) { ds_P = b.P; ds_n = b.n; }
  TT_REQUIRE(b.P == ds_P && b.n == ds_n, "dataset blocks must share probe count and block size");
  const long take = std::min<long>(b.N, cap - ds_N);
  if (take <= 0) return;
  const long need = ds_N + take;
  if (need > ds_cap) {
    const long nc = std::max<long>(need, 2 * ds_cap);
    auto grow = [&](FBuf& buf, long per) {
      FBuf nb((size_t)nc * per);
      if (ds_N > 0)
        TT_HIP(hipMemcpyAsync(nb.get(), buf.get(), sizeof(float) * ds_N * per, hipMemcpyDeviceToDevice, c.s));
      c.sync();
      buf = std::move(nb);
    };
    grow(dsF, in);
    grow(dsR, (long)ds_P * ds_n);
    grow(dsY, (long)ds_P * ds_n);
    grow(dsS, 1);
    grow(dsW, ds_P);
    ds_cap = nc;
  }
  auto put = [&](FBuf& dst, const float* src, long per) {
    TT_HIP(hipMemcpyAsync(dst.get() + ds_N * per, src, sizeof(float) * take * per, hipMemcpyDeviceToDevice, c.s));
  };
  put(dsF, b.F, in);
  put(dsR, b.R, (long)ds_P * ds_n);
  put(dsY, b.Y, (long)ds_P * ds_n);
  put(dsS, b.S, 1);
  put(dsW, b.W, ds_P);
  c.sync();
  ds_N += take;
}

void mlp_train(Mlp& net, const MlpBatch& data, int epochs, int batch, float lr, unsigned long long seed,
               std::vector<double>& hist, Ctx& c) {
  const long N = data.N;
  const int per_rn = data.P * data.n;
  batch = (int)std::max<long>(1, std::min<long>(batch, N));
  std::mt19937_64 rng(seed);
  std::vector<int> perm(N);
  for (long i = 0; i < N; ++i) perm[i] = (int)i;
  DevBuf idx((size_t)(batch + 1) / 2);
  FBuf F((size_t)batch * net.in), R((size_t)batch * per_rn), Y((size_t)batch * per_rn), S(batch), W((size_t)batch * data.P);
  hist.clear();
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    double acc = 0.0;
    long seen = 0;
    for (long b0 = 0; b0 + batch <= N; b0 += batch) {
      TT_HIP(hipMemcpyAsync(idx.get(), perm.data() + b0, sizeof(int) * batch, hipMemcpyHostToDevice, c.s));
      const int* ip = reinterpret_cast<const int*>(idx.get());
      auto g = [&](const float* src, long per, FBuf& dst) {
        hipLaunchKernelGGL(gather_rows_kernel, dim3(nblocks((size_t)batch * per, 256)), dim3(256), 0, c.s, src, ip,
                           (long)batch, per, dst.get());
      };
      g(data.F, net.in, F);
      g(data.R, per_rn, R);
      g(data.Y, per_rn, Y);
      g(data.S, 1, S);
      g(data.W, data.P, W);
      TT_HIP(hipGetLastError());
      MlpBatch mb{batch, data.P, data.n, F.get(), R.get(), Y.get(), S.get(), W.get()};
      const double l = net.loss_grad(mb, c);
      net.adam_step(lr, c);
      acc += l * batch;
      seen += batch;
    }
    hist.push_back(seen ? acc / seen : 0.0);
  }
  c.sync();
}

void mlp_block_data(const BlockJacobi& raw, const BlockJacobi& inv, const std::function<void(const double*, double*)>& apply_K,
                    const float ctx[4], int nprobe, unsigned long long seed, FBuf& F, FBuf& R, FBuf& Y, FBuf& S,
                    FBuf& W, Ctx& c) {
  const int n = raw.L * raw.m;
  const long nb = (long)raw.r * raw.s;
  const long len = (long)raw.L * raw.r * raw.m * raw.s;
  F.reserve((size_t)nb * (n * n + 5));
  S.reserve(nb);
  R.reserve((size_t)nb * nprobe * n);
  Y.reserve((size_t)nb * nprobe * n);
  W.reserve((size_t)nb * nprobe);
  FBuf cdev(4);
  TT_HIP(hipMemcpyAsync(cdev.get(), ctx, sizeof(float) * 4, hipMemcpyHostToDevice, c.s));
  hipLaunchKernelGGL(block_features_kernel, dim3(nblocks(nb, 64)), dim3(64), 0, c.s, raw.blk.get(), (int)nb, n,
                     cdev.get(), F.get(), S.get());
  DevBuf x(len), y(len);
  for (int p = 0; p < nprobe; ++p) {
    hipLaunchKernelGGL(normal_kernel, dim3(nblocks(len, 256)), dim3(256), 0, c.s, x.get(), len,
                       seed * 1315423911ull + (unsigned long long)p);
    apply_K(x.get(), y.get());
    // weight: nb / |x|^2 (the loss is then the mean block share of |x - M K x|^2 / |x|^2)
    const double nx = dev_norm(x.get(), len, c);
    const float w = (float)(nb / std::max(nx * nx, 1e-300));
    hipLaunchKernelGGL(probe_kernel, dim3(nblocks(nb * n, 256)), dim3(256), 0, c.s, inv.blk.get(), x.get(), y.get(),
                       raw.r, raw.m, raw.s, raw.L, nprobe, p, w, R.get(), Y.get(), W.get());
    TT_HIP(hipGetLastError());
  }
  c.sync();
}

void mlp_correct_blocks(Mlp& net, const BlockJacobi& raw, BlockJacobi& inv, const float ctx[4], Ctx& c) {
  const int n = raw.L * raw.m;
  const long nb = (long)raw.r * raw.s;
  TT_REQUIRE(net.in == n * n + 5 && net.out == n * n, "network dimensions do not match the local blocks");
  FBuf F((size_t)nb * (n * n + 5)), S(nb), o((size_t)nb * n * n), cdev(4);
  TT_HIP(hipMemcpyAsync(cdev.get(), ctx, sizeof(float) * 4, hipMemcpyHostToDevice, c.s));
  hipLaunchKernelGGL(block_features_kernel, dim3(nblocks(nb, 64)), dim3(64), 0, c.s, raw.blk.get(), (int)nb, n,
                     cdev.get(), F.get(), S.get());
  net.forward(F.get(), (int)nb, o.get(), c);
  hipLaunchKernelGGL(add_correction_kernel, dim3(nblocks(nb * n * n, 256)), dim3(256), 0, c.s, inv.blk.get(), o.get(),
                     S.get(), nb, n);
  TT_HIP(hipGetLastError());
  c.sync();
}

}  // namespace ttipm
