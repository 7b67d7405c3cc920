// Strided, batched GEMM on the CDNA4 matrix cores.
//
// Every contraction of the TT method (environment builds, the projected local
// products, dense local blocks, the rounding's small products) reduces to
//     C[b] = alpha * A[b] * B[b] + beta * C[b]
// with arbitrary element strides, so one kernel family serves them all.
//
//  * FP64: v_mfma_f64_16x16x4f64.  A 256-thread workgroup (four 64-lane waves in
//    a 2 x 2 arrangement) owns a 64 x 64 output tile; each wave owns 32 x 32,
//    i.e. 2 x 2 MFMA tiles of 16 x 16 with independent accumulators.  Tiles of A
//    (64 x 16) and B (16 x 64) are staged through LDS in k-major order so that a
//    lane reads its MFMA operand (row lane%16, k lane/16) with one LDS load.
//    The global -> LDS copy maps threads along whichever index is unit-stride,
//    so loads coalesce for both transposed and plain operands.
//  * Mixed precision: the same tiling with v_mfma_f32_16x16x32_bf16 — operands
//    rounded to BF16 on the way into LDS, FP32 accumulation, FP32 or FP64 out.
//  * Split-K for tall-K, small-MN products (the last stage of a local product
//    has K = R' r' up to 32k but only r*4 x r outputs): each K slice writes its
//    partial tile to a workspace, and a second kernel reduces the slices in a
//    fixed order, so results are bit-reproducible run to run.
#include "gemm.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <vector>

namespace ttipm {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int PADF = 17;   // FP64 tiled kernel

struct KArgs {
  int M, N, K;
  int kslices, kchunk;      // split-K: slice s covers k in [s*kchunk, min(K,(s+1)*kchunk))
  const double* A; long am, ak, sA;
  const double* B; long bk, bn, sB;
  double* C; long cm, cn, sC;
  double alpha, beta;
  double* P;                // split-K partials [batch][kslices][M][N] (dense)
};

// Result layouts of the 16 x 16 MFMA tiles (measured on gfx950): every lane
// holds column lane%16; the four accumulator values are rows lane/16 + 4e for
// v_mfma_f64_16x16x4f64 and rows 4*(lane/16) + e for v_mfma_f32_16x16x32_bf16.

// FP64 kernel, templated on the MFMA tiles per wave (WM x WN of 16 x 16; the
// workgroup tile is (32 WM) x (32 WN)) and on which operand index is unit
// stride (AKC: A is k-contiguous, BKC: B is k-contiguous), so that the copy
// pattern is fixed at compile time.  Every thread owns NA elements of each A
// tile and NB of each B tile at fixed (row, k) positions; their 32-bit element
// offsets are computed once, so a k-step costs one uniform pointer bump plus
// one load per element.  Rows or columns past the matrix edge are clamped to
// the last valid one (no divergent branches in the loop); only a ragged last
// k-step checks k.  The next k-tile is fetched into
// registers while the current one is consumed from LDS (two LDS buffers, one
// barrier per k-step).  The register budget is capped at two waves per SIMD
// (256 VGPR + AGPR): a second wave hides the first one's LDS and barrier
// stalls, which measured faster than one wave with more prefetch registers.
// Workgroups are dispatched round-robin over the eight
// XCDs; tiles are renumbered so that each XCD works on a contiguous run of
// output tiles (shared A row panels and B column panels stay in its L2).
// One output tile (tm, tn) of batch entry bidx, K slice `slice`.
template <int WM, int WN, bool AKC, bool BKC>
__device__ __forceinline__ void gemm_f64_tile(const KArgs& g, int tm, int tn, int bidx, int slice) {
  constexpr int TM = 32 * WM, TN = 32 * WN;
  constexpr int NA = TM * BK / 256, NB = BK * TN / 256;
  // element e of a thread sits at (fixed, base + STEP * e) along (m, k) or (k, m)
  constexpr int ASTEP = AKC ? 256 / BK : 256 / TM;
  constexpr int BSTEP = BKC ? 256 / BK : 256 / TN;
  // Row pitch TM + 17 doubles: the two half-waves of an operand read (rows kr
  // and kr + 1) start 34 banks apart, and the transposing k-contiguous stores
  // of one row of 16 threads land on 16 distinct bank pairs (34 k mod 64).
  __shared__ double As[2][BK][TM + PADF];
  __shared__ double Bs[2][BK][TN + PADF];
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;
  const int m0 = tm * TM, n0 = tn * TN;
  const int kbeg = slice * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
  const double* A = g.A + (long)bidx * g.sA;
  const double* B = g.B + (long)bidx * g.sB;
  // tile positions of this thread's elements
  const int a_mt = AKC ? tid / BK : tid % TM;   // m of element 0
  const int a_kt = AKC ? tid % BK : tid / TM;   // k of element 0
  const int b_nt = BKC ? tid / BK : tid % TN;
  const int b_kt = BKC ? tid % BK : tid / TN;
  // Rows of A past M (columns of B past N) are clamped to the last valid one:
  // they only feed output rows (columns) that the epilogue never stores, so
  // they need no masking.  Only k past the end must contribute zero.
  // Byte offsets (32-bit) from the uniform k-step base pointer: the loads
  // then take the scalar-base + vector-offset form with no 64-bit VALU math.
  unsigned offA[NA], offB[NB];
#pragma unroll
  for (int e = 0; e < NA; ++e) {
    const int m = m0 + a_mt + (AKC ? ASTEP * e : 0), k = a_kt + (AKC ? 0 : ASTEP * e);
    offA[e] = 8u * (unsigned)(min(m, g.M - 1) * (int)g.am + k * (int)g.ak);
  }
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int n = n0 + b_nt + (BKC ? BSTEP * e : 0), k = b_kt + (BKC ? 0 : BSTEP * e);
    offB[e] = 8u * (unsigned)(min(n, g.N - 1) * (int)g.bn + k * (int)g.bk);
  }
  double ra[NA], rb[NB];
  // Full k-steps load without any select, so the loads stay in flight across
  // the MFMA block and are first waited on when stashed into LDS.
  auto fetch = [&](int k0) {
    const char* Ak = reinterpret_cast<const char*>(A + (long)k0 * g.ak);
    const char* Bk = reinterpret_cast<const char*>(B + (long)k0 * g.bk);
    if (k0 + BK <= kend) {
#pragma unroll
      for (int e = 0; e < NA; ++e) ra[e] = *reinterpret_cast<const double*>(Ak + offA[e]);
#pragma unroll
      for (int e = 0; e < NB; ++e) rb[e] = *reinterpret_cast<const double*>(Bk + offB[e]);
    } else {
      // ragged last k-step: clamp k to the last valid index and zero it
#pragma unroll
      for (int e = 0; e < NA; ++e) {
        const int k = a_kt + (AKC ? 0 : ASTEP * e);
        const int kc = min(k, kend - 1 - k0);
        const double v = *reinterpret_cast<const double*>(Ak + offA[e] + 8L * (kc - k) * g.ak);
        ra[e] = (k0 + k < kend) ? v : 0.0;
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int k = b_kt + (BKC ? 0 : BSTEP * e);
        const int kc = min(k, kend - 1 - k0);
        const double v = *reinterpret_cast<const double*>(Bk + offB[e] + 8L * (kc - k) * g.bk);
        rb[e] = (k0 + k < kend) ? v : 0.0;
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int m = a_mt + (AKC ? ASTEP * e : 0), k = a_kt + (AKC ? 0 : ASTEP * e);
      As[buf][k][m] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int n = b_nt + (BKC ? BSTEP * e : 0), k = b_kt + (BKC ? 0 : BSTEP * e);
      Bs[buf][k][n] = rb[e];
    }
  };
  f64x4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  int buf = 0;
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + lane / 16;
      double a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = As[buf][kr][wm * (16 * WM) + i * 16 + (lane % 16)];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Bs[buf][kr][wn * (16 * WN) + j * 16 + (lane % 16)];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // epilogue: f64 MFMA result rows lane/16 + 4e, column lane%16
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * (16 * WM) + i * 16 + (lane / 16) + 4 * e;
        const int col = n0 + wn * (16 * WN) + j * 16 + (lane % 16);
        if (row < g.M && col < g.N) {
          const double v = acc[i][j][e];
          if (g.kslices > 1) {
            g.P[(((long)bidx * g.kslices + slice) * g.M + row) * g.N + col] = v;
          } else {
            double* c = g.C + (long)bidx * g.sC + (long)row * g.cm + (long)col * g.cn;
            *c = (g.beta == 0.0) ? g.alpha * v : g.alpha * v + g.beta * (*c);
          }
        }
      }
}

template <int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f64_kernel(KArgs g) {
  // XCD-aware renumbering of the (m, n) tile grid
  const int gmt = gridDim.x, gnt = gridDim.y;
  const int tiles = gmt * gnt;
  const int lin = blockIdx.y * gmt + blockIdx.x;
  int t = lin;
  if (tiles >= 16) {
    const int per = (tiles + 7) / 8;
    const int cand = (lin % 8) * per + lin / 8;
    // keep the map a bijection when tiles is not a multiple of 8
    t = (tiles % 8 == 0) ? cand : lin;
  }
  gemm_f64_tile<WM, WN, AKC, BKC>(g, t / gnt, t % gnt, blockIdx.z / g.kslices, blockIdx.z % g.kslices);
}

// Several independent products in one launch: problem i owns the workgroups
// [end[i-1], end[i]) of a 1-D grid, tiles * batch * kslices of them.  A
// projected local product applies several operators to the same block
// vector; each stage of all of them then costs one launch whose workgroups
// run side by side instead of one small launch per operator.
constexpr int kMaxGroup = 8;
struct GroupArgs {
  KArgs g[kMaxGroup];
  int end[kMaxGroup];       // prefix sums of the workgroup counts
  int gn[kMaxGroup];        // tile columns of each problem
  int tiles[kMaxGroup];     // output tiles of each problem
  int n;
};

// problem, output tile, batch entry and K slice of this workgroup
struct GroupTile {
  int i, tm, tn, bidx, slice;
};
__device__ __forceinline__ GroupTile group_tile(const GroupArgs& ga) {
  const int lin = blockIdx.x;
  int i = 0;
  while (i + 1 < ga.n && lin >= ga.end[i]) ++i;
  const int local = lin - (i ? ga.end[i - 1] : 0);
  const int ks = ga.g[i].kslices;
  const int t = local % ga.tiles[i], z = local / ga.tiles[i];
  return {i, t / ga.gn[i], t % ga.gn[i], z / ks, z % ks};
}

template <int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f64_grouped_kernel(GroupArgs ga) {
  const GroupTile q = group_tile(ga);
  gemm_f64_tile<WM, WN, AKC, BKC>(ga.g[q.i], q.tm, q.tn, q.bidx, q.slice);
}

// Small products (both output dimensions <= 64, short K: the frames of rank
// <= 16): one wave per 16 x 16 output block, operands loaded from global
// memory (L2) straight into the MFMA operand registers, no LDS and no
// barrier.  Lane l supplies row l%16 of A and column l%16 of B at k = 4u +
// l/16 of each group of 16 k, exactly as the tiled kernel reads them from LDS,
// so the MFMA sequence of every accumulator (k ascending in steps of 4, a
// ragged tail padded with zeros) and hence every result is bit-identical to
// the tiled kernel without split-K.  Two groups of 16 k (eight loads per
// operand) are issued before their MFMAs.
__device__ __forceinline__ void gemm_f64_block16(const KArgs& g, int bm, int bn, int bidx) {
  const int lane = threadIdx.x % 64, q = lane / 16, r16 = lane % 16;
  const int m0 = bm * 16, n0 = bn * 16;
  const int row = min(m0 + r16, g.M - 1), col = min(n0 + r16, g.N - 1);
  const double* Ar = g.A + (long)bidx * g.sA + (long)row * g.am;
  const double* Bc = g.B + (long)bidx * g.sB + (long)col * g.bn;
  const long ak = g.ak, bk = g.bk;
  f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
  int k0 = 0;
  for (; k0 + 32 <= g.K; k0 += 32) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = Ar[(long)(k0 + 4 * u + q) * ak];
      b[u] = Bc[(long)(k0 + 4 * u + q) * bk];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
  // the rest (< 32 k): all loads first (k clamped, zeros past K), then one
  // MFMA per group of four k that holds any k < K (a group of the tiled
  // kernel whose MFMAs see only zeros leaves the accumulator unchanged)
  if (k0 < g.K) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + 4 * u + q;
      const bool in = k < g.K;
      const int kc = in ? k : g.K - 1;
      const double av = Ar[(long)kc * ak], bv = Bc[(long)kc * bk];
      a[u] = in ? av : 0.0;
      b[u] = in ? bv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + 4 * u < g.K) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int rr = m0 + q + 4 * e, cc = n0 + r16;
    if (rr < g.M && cc < g.N) {
      double* c = g.C + (long)bidx * g.sC + (long)rr * g.cm + (long)cc * g.cn;
      *c = (g.beta == 0.0) ? g.alpha * acc[e] : g.alpha * acc[e] + g.beta * (*c);
    }
  }
}

// blocks: 16 x 16 output blocks of one batch entry (gn columns of them); one
// wave each, four waves per workgroup
__global__ __launch_bounds__(256) void gemm_f64_small_kernel(KArgs g, int gn, int blocks, long total) {
  const long w = (long)blockIdx.x * 4 + threadIdx.x / 64;
  if (w >= total) return;
  const int t = (int)(w % blocks), bidx = (int)(w / blocks);
  gemm_f64_block16(g, t / gn, t % gn, bidx);
}

// Grouped small products: problem i owns the waves [end[i-1], end[i]),
// tiles[i] 16 x 16 blocks (gn[i] columns of them) per batch entry.
__global__ __launch_bounds__(256) void gemm_f64_small_grouped_kernel(GroupArgs ga) {
  const int w = blockIdx.x * 4 + threadIdx.x / 64;
  if (w >= ga.end[ga.n - 1]) return;
  int i = 0;
  while (i + 1 < ga.n && w >= ga.end[i]) ++i;
  const int local = w - (i ? ga.end[i - 1] : 0);
  const int t = local % ga.tiles[i], bidx = local / ga.tiles[i];
  gemm_f64_block16(ga.g[i], t / ga.gn[i], t % ga.gn[i], bidx);
}

// BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16): lane l supplies
// row l%16 and the eight k-values 8(l/16)..8(l/16)+7 of each operand, so the
// LDS tiles are stored with k contiguous ([m][k], row pitch 40 values = 80
// bytes) and each operand is one 16-byte LDS read; the 16 rows of a read start
// on distinct 4-bank groups.  FP64 operands are fetched with the same
// precomputed-offset scheme as the FP64 kernel (loads in flight across the
// MFMA block) and rounded to BF16 when stashed into LDS; BK = 32 is one MFMA
// k-depth.  Accumulators are FP32; the epilogue writes FP64.
constexpr int BK16 = 32;
constexpr int P16 = 40;   // LDS row pitch in bf16 values

template <int WM, int WN, bool AKC, bool BKC>
__device__ __forceinline__ void gemm_bf16_tile(const KArgs& g, int tm, int tn, int bidx, int slice) {
  constexpr int TM = 32 * WM, TN = 32 * WN;
  constexpr int NA = TM * BK16 / 256, NB = BK16 * TN / 256;
  constexpr int ASTEP = AKC ? 256 / BK16 : 256 / TM;
  constexpr int BSTEP = BKC ? 256 / BK16 : 256 / TN;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][P16];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TN][P16];
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;
  const int m0 = tm * TM, n0 = tn * TN;
  const int kbeg = slice * g.kchunk, kend = min(g.K, kbeg + g.kchunk);
  const double* A = g.A + (long)bidx * g.sA;
  const double* B = g.B + (long)bidx * g.sB;
  const int a_mt = AKC ? tid / BK16 : tid % TM;
  const int a_kt = AKC ? tid % BK16 : tid / TM;
  const int b_nt = BKC ? tid / BK16 : tid % TN;
  const int b_kt = BKC ? tid % BK16 : tid / TN;
  unsigned offA[NA], offB[NB];
#pragma unroll
  for (int e = 0; e < NA; ++e) {
    const int m = m0 + a_mt + (AKC ? ASTEP * e : 0), k = a_kt + (AKC ? 0 : ASTEP * e);
    offA[e] = 8u * (unsigned)(min(m, g.M - 1) * (int)g.am + k * (int)g.ak);
  }
#pragma unroll
  for (int e = 0; e < NB; ++e) {
    const int n = n0 + b_nt + (BKC ? BSTEP * e : 0), k = b_kt + (BKC ? 0 : BSTEP * e);
    offB[e] = 8u * (unsigned)(min(n, g.N - 1) * (int)g.bn + k * (int)g.bk);
  }
  double ra[NA], rb[NB];
  auto fetch = [&](int k0) {
    const char* Ak = reinterpret_cast<const char*>(A + (long)k0 * g.ak);
    const char* Bk = reinterpret_cast<const char*>(B + (long)k0 * g.bk);
    if (k0 + BK16 <= kend) {
#pragma unroll
      for (int e = 0; e < NA; ++e) ra[e] = *reinterpret_cast<const double*>(Ak + offA[e]);
#pragma unroll
      for (int e = 0; e < NB; ++e) rb[e] = *reinterpret_cast<const double*>(Bk + offB[e]);
    } else {
#pragma unroll
      for (int e = 0; e < NA; ++e) {
        const int k = a_kt + (AKC ? 0 : ASTEP * e);
        const int kc = min(k, kend - 1 - k0);
        const double v = *reinterpret_cast<const double*>(Ak + offA[e] + 8L * (kc - k) * g.ak);
        ra[e] = (k0 + k < kend) ? v : 0.0;
      }
#pragma unroll
      for (int e = 0; e < NB; ++e) {
        const int k = b_kt + (BKC ? 0 : BSTEP * e);
        const int kc = min(k, kend - 1 - k0);
        const double v = *reinterpret_cast<const double*>(Bk + offB[e] + 8L * (kc - k) * g.bk);
        rb[e] = (k0 + k < kend) ? v : 0.0;
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < NA; ++e) {
      const int m = a_mt + (AKC ? ASTEP * e : 0), k = a_kt + (AKC ? 0 : ASTEP * e);
      As[buf][m][k] = (__bf16)ra[e];
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int n = b_nt + (BKC ? BSTEP * e : 0), k = b_kt + (BKC ? 0 : BSTEP * e);
      Bs[buf][n][k] = (__bf16)rb[e];
    }
  };
  f32x4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int buf = 0;
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  const int kq = 8 * (lane / 16);
  for (int k0 = kbeg; k0 < kend; k0 += BK16) {
    const bool more = k0 + BK16 < kend;
    if (more) fetch(k0 + BK16);
    bf16x8 a[WM], b[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * (16 * WM) + i * 16 + (lane % 16)][kq]);
#pragma unroll
    for (int j = 0; j < WN; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * (16 * WN) + j * 16 + (lane % 16)][kq]);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // epilogue: rows 4(lane/16) + e, column lane%16 of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * (16 * WM) + i * 16 + 4 * (lane / 16) + e;
        const int col = n0 + wn * (16 * WN) + j * 16 + (lane % 16);
        if (row < g.M && col < g.N) {
          const double v = (double)acc[i][j][e];
          if (g.kslices > 1) {
            g.P[(((long)bidx * g.kslices + slice) * g.M + row) * g.N + col] = v;
          } else {
            double* c = g.C + (long)bidx * g.sC + (long)row * g.cm + (long)col * g.cn;
            *c = (g.beta == 0.0) ? g.alpha * v : g.alpha * v + g.beta * (*c);
          }
        }
      }
}

template <int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16_kernel(KArgs g) {
  const int gmt = gridDim.x, gnt = gridDim.y;
  const int tiles = gmt * gnt;
  const int lin = blockIdx.y * gmt + blockIdx.x;
  int t = lin;
  if (tiles >= 16) {
    const int per = (tiles + 7) / 8;
    const int cand = (lin % 8) * per + lin / 8;
    t = (tiles % 8 == 0) ? cand : lin;
  }
  gemm_bf16_tile<WM, WN, AKC, BKC>(g, t / gnt, t % gnt, blockIdx.z / g.kslices, blockIdx.z % g.kslices);
}

template <int WM, int WN, bool AKC, bool BKC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16_grouped_kernel(GroupArgs ga) {
  const GroupTile q = group_tile(ga);
  gemm_bf16_tile<WM, WN, AKC, BKC>(ga.g[q.i], q.tm, q.tn, q.bidx, q.slice);
}

__device__ __forceinline__ void splitk_reduce_one(const KArgs& g, long idx) {
  int b = (int)(idx / ((long)g.M * g.N));
  long rem = idx % ((long)g.M * g.N);
  int row = (int)(rem / g.N), col = (int)(rem % g.N);
  // eight independent partial sums keep eight loads in flight per thread; the
  // association is fixed, so results are reproducible run to run
  const long stride = (long)g.M * g.N;
  const double* p = g.P + (long)b * g.kslices * stride + rem;
  double part[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int sl = 0;
  for (; sl + 8 <= g.kslices; sl += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) part[u] += p[(long)(sl + u) * stride];
  }
  for (; sl < g.kslices; ++sl) part[0] += p[(long)sl * stride];
  const double s = ((part[0] + part[1]) + (part[2] + part[3])) + ((part[4] + part[5]) + (part[6] + part[7]));
  double* c = g.C + (long)b * g.sC + (long)row * g.cm + (long)col * g.cn;
  *c = (g.beta == 0.0) ? g.alpha * s : g.alpha * s + g.beta * (*c);
}

__global__ void splitk_reduce_kernel(KArgs g, int batch) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)batch * g.M * g.N;
  if (idx >= total) return;
  splitk_reduce_one(g, idx);
}

// Reduce of the split problems of a grouped launch: problem i owns outputs
// [end[i-1], end[i]) of a 1-D index space (`end` holds output, not workgroup,
// counts here; unsplit problems own none).
__global__ void splitk_reduce_grouped_kernel(GroupArgs ga) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ga.end[ga.n - 1]) return;
  int i = 0;
  while (i + 1 < ga.n && idx >= ga.end[i]) ++i;
  splitk_reduce_one(ga.g[i], idx - (i ? ga.end[i - 1] : 0));
}

__global__ void scale_c_kernel(double* C, long cm, long cn, long sC, int M, int N, int batch, double beta) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)batch * M * N;
  if (idx >= total) return;
  int b = (int)(idx / ((long)M * N));
  long rem = idx % ((long)M * N);
  int row = (int)(rem / N), col = (int)(rem % N);
  double* c = C + (long)b * sC + (long)row * cm + (long)col * cn;
  *c = (beta == 0.0) ? 0.0 : beta * (*c);
}

static Workspace g_default_ws;

double* Workspace::take(size_t n) {
  if (fixed) {
    if (n > fixed_n) throw Error(TT_ERR_ARG, "split-K partials exceed the fixed workspace");
    return fixed;
  }
  buf.reserve(n);
  return buf.get();
}

// Slice count of the split-K rule for `tiles` output tiles.
static int splitk_slices(long tiles, int K, int kstep) {
  int ks = 1;
  if (tiles < 128 && K >= 16 * kstep) {
    ks = (int)std::min<long>((256 + tiles - 1) / tiles, (long)K / (8 * kstep));
    ks = std::max(1, std::min(ks, 64));
  }
  int chunk = (K + ks - 1) / ks;
  chunk = ((chunk + kstep - 1) / kstep) * kstep;
  return (K + chunk - 1) / chunk;
}

size_t gemm_splitk_need(const Gemm& q, GemmPrec prec) {
  if (q.M <= 0 || q.N <= 0 || q.batch <= 0 || q.K <= 0) return 0;
  const int kstep = (prec == GemmPrec::BF16) ? BK16 : BK;
  // the single launch picks tiles of at least 64 x 64, the grouped one 64 x 64:
  // 64 x 64 tiles give the most output tiles and the fewest slices, 128 x 128
  // the fewest tiles and the most slices; both bound the slice count
  size_t need = 0;
  for (int t = 64; t <= 128; t *= 2) {
    const long tiles = (long)((q.M + t - 1) / t) * ((q.N + t - 1) / t) * q.batch;
    const int ks = splitk_slices(tiles, q.K, kstep);
    if (ks > 1) need = std::max(need, (size_t)q.batch * ks * q.M * q.N);
  }
  return need;
}

// Products small enough for the register-direct kernel: both output
// dimensions within one 64 x 64 tile and K short enough that the tiled kernel
// would not split it.
static bool small_gemm(const Gemm& q, GemmPrec prec) {
  return prec == GemmPrec::F64 && q.M <= 64 && q.N <= 64 && q.K < 16 * BK;
}

template <int WM, int WN>
void launch_bf16(dim3 grid, hipStream_t stream, const KArgs& g, double flops, double bytes) {
  const bool akc = (g.ak == 1), bkc = (g.bk == 1 && g.bn != 1);
  if (akc && bkc)
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_kernel<WM, WN, true, true>, grid, dim3(256), 0u, stream, g);
  else if (akc)
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_kernel<WM, WN, true, false>, grid, dim3(256), 0u, stream, g);
  else if (bkc)
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_kernel<WM, WN, false, true>, grid, dim3(256), 0u, stream, g);
  else
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_kernel<WM, WN, false, false>, grid, dim3(256), 0u, stream, g);
}

template <int WM, int WN>
void launch_f64(dim3 grid, hipStream_t stream, const KArgs& g, double flops, double bytes) {
  const bool akc = (g.ak == 1), bkc = (g.bk == 1 && g.bn != 1);
  if (akc && bkc)
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_kernel<WM, WN, true, true>, grid, dim3(256), 0u, stream, g);
  else if (akc)
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_kernel<WM, WN, true, false>, grid, dim3(256), 0u, stream, g);
  else if (bkc)
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_kernel<WM, WN, false, true>, grid, dim3(256), 0u, stream, g);
  else
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_kernel<WM, WN, false, false>, grid, dim3(256), 0u, stream, g);
}

void gemm(const Gemm& q, hipStream_t stream, Workspace* ws, GemmPrec prec) {
  if (q.M <= 0 || q.N <= 0 || q.batch <= 0) return;
  if (q.K <= 0) {  // C = beta C
    long total = (long)q.batch * q.M * q.N;
    hipLaunchKernelGGL(scale_c_kernel, dim3(nblocks(total, 256)), dim3(256), 0, stream, q.C, q.cm, q.cn,
                       q.sC, q.M, q.N, q.batch, q.beta);
    TT_HIP(hipGetLastError());
    return;
  }
  // the FP64 kernel addresses operands with 32-bit byte offsets from the
  // (64-bit) batch and k-step base; strides are non-negative for every caller
  if (q.am < 0 || q.ak < 0 || q.bk < 0 || q.bn < 0 ||
      (double)(q.M - 1) * q.am + (double)(q.K - 1 + BK16) * q.ak > 536870911.0 ||
      (double)(q.N - 1) * q.bn + (double)(q.K - 1 + BK16) * q.bk > 536870911.0)
    throw Error(TT_ERR_ARG, "gemm operand too large for 32-bit byte offsets (M " + std::to_string(q.M) + " N " +
                                std::to_string(q.N) + " K " + std::to_string(q.K) + " am " + std::to_string(q.am) +
                                " ak " + std::to_string(q.ak) + " bk " + std::to_string(q.bk) + " bn " +
                                std::to_string(q.bn) + " batch " + std::to_string(q.batch) + ")");
  KArgs g;
  g.M = q.M; g.N = q.N; g.K = q.K;
  g.A = q.A; g.am = q.am; g.ak = q.ak; g.sA = q.sA;
  g.B = q.B; g.bk = q.bk; g.bn = q.bn; g.sB = q.sB;
  g.C = q.C; g.cm = q.cm; g.cn = q.cn; g.sC = q.sC;
  g.alpha = q.alpha; g.beta = q.beta;
  if (small_gemm(q, prec)) {
    g.kslices = 1;
    g.kchunk = q.K;
    g.P = nullptr;
    const int gm = (q.M + 15) / 16, gn = (q.N + 15) / 16;
    const long total = (long)gm * gn * q.batch;
    const double flops = 2.0 * q.M * q.N * (double)q.K * q.batch;
    const double bytes =
        8.0 * q.batch * ((double)q.M * q.K + (double)q.K * q.N + (double)q.M * q.N * (q.beta != 0.0 ? 2 : 1));
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_small_kernel, dim3((unsigned)((total + 3) / 4)), dim3(256), 0u,
                stream, g, gn, gm * gn, total);
    TT_HIP(hipGetLastError());
    return;
  }
  // Tile shape (both precisions): 128 x 128 for large outputs, 128 x 64 /
  // 64 x 128 for skinny ones, 64 x 64 otherwise.
  // The largest tile that still gives the chip enough workgroups (min_tiles,
  // default two per CU so that two waves share each SIMD and hide each other's
  // LDS and global latency) and does not overhang a dimension shorter than
  // the tile; else 64 x 64.  TTIPM_GEMM_MIN_TILES overrides the threshold.
  static const long min_tiles = [] {
    const char* e = std::getenv("TTIPM_GEMM_MIN_TILES");
    const long v = e ? std::atol(e) : 0;
    return v > 0 ? v : 512L;
  }();
  int TMs = BM, TNs = BN;
  {
    const int cand[3][2] = {{128, 128}, {128, 64}, {64, 128}};
    for (const auto& t : cand) {
      if (q.M < t[0] || q.N < t[1]) continue;
      const long nt = (long)((q.M + t[0] - 1) / t[0]) * ((q.N + t[1] - 1) / t[1]) * q.batch;
      if (nt >= min_tiles) { TMs = t[0]; TNs = t[1]; break; }
    }
  }
  const int gm = (q.M + TMs - 1) / TMs, gn = (q.N + TNs - 1) / TNs;
  const long tiles = (long)gm * gn * q.batch;
  // Split K only when the output tiles cannot occupy half of the 256 CUs and K
  // is long: every slice writes a full partial tile that the reduce kernel
  // reads back, so the slice count is kept to what fills the chip.
  int ks = 1;
  const int kstep = (prec == GemmPrec::BF16) ? BK16 : BK;
  if (tiles < 128 && q.K >= 16 * kstep) {
    ks = (int)std::min<long>((256 + tiles - 1) / tiles, (long)q.K / (8 * kstep));
    ks = std::max(1, std::min(ks, 64));
  }
  g.kslices = ks;
  int chunk = (q.K + ks - 1) / ks;
  chunk = ((chunk + kstep - 1) / kstep) * kstep;
  g.kchunk = chunk;
  ks = (q.K + chunk - 1) / chunk;
  g.kslices = ks;
  g.P = nullptr;
  if (ks > 1) {
    Workspace* w = ws ? ws : &g_default_ws;
    size_t need = (size_t)q.batch * ks * q.M * q.N;
    g.P = w->take(need);
  }
  dim3 grid(gm, gn, q.batch * ks);
  const double flops = 2.0 * q.M * q.N * (double)q.K * q.batch;
  const double bytes = 8.0 * q.batch * ((double)q.M * q.K + (double)q.K * q.N + (double)q.M * q.N * (q.beta != 0.0 ? 2 : 1));
  if (prec == GemmPrec::BF16) {
    if (TMs == 128 && TNs == 128)
      launch_bf16<4, 4>(grid, stream, g, flops, bytes);
    else if (TMs == 128)
      launch_bf16<4, 2>(grid, stream, g, flops, bytes);
    else if (TNs == 128)
      launch_bf16<2, 4>(grid, stream, g, flops, bytes);
    else
      launch_bf16<2, 2>(grid, stream, g, flops, bytes);
  } else if (TMs == 128 && TNs == 128)
    launch_f64<4, 4>(grid, stream, g, flops, bytes);
  else if (TMs == 128)
    launch_f64<4, 2>(grid, stream, g, flops, bytes);
  else if (TNs == 128)
    launch_f64<2, 4>(grid, stream, g, flops, bytes);
  else
    launch_f64<2, 2>(grid, stream, g, flops, bytes);
  TT_HIP(hipGetLastError());
  if (ks > 1) {
    long total = (long)q.batch * q.M * q.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(nblocks(total, 256)), dim3(256), 0, stream, g, q.batch);
    TT_HIP(hipGetLastError());
  }
}

template <int WM, int WN>
void launch_bf16_grouped(int blocks, hipStream_t stream, const GroupArgs& ga, bool akc, bool bkc, double flops,
                         double bytes) {
  const dim3 grid(blocks), blk(256);
  if (akc && bkc)
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_grouped_kernel<WM, WN, true, true>, grid, blk, 0u, stream, ga);
  else if (akc)
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_grouped_kernel<WM, WN, true, false>, grid, blk, 0u, stream, ga);
  else if (bkc)
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_grouped_kernel<WM, WN, false, true>, grid, blk, 0u, stream, ga);
  else
    launch_prof(PK_GEMM_BF16, flops, bytes, gemm_bf16_grouped_kernel<WM, WN, false, false>, grid, blk, 0u, stream,
                ga);
}

template <int WM, int WN>
void launch_f64_grouped(int blocks, hipStream_t stream, const GroupArgs& ga, bool akc, bool bkc, double flops,
                        double bytes) {
  const dim3 grid(blocks), blk(256);
  if (akc && bkc)
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_grouped_kernel<WM, WN, true, true>, grid, blk, 0u, stream, ga);
  else if (akc)
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_grouped_kernel<WM, WN, true, false>, grid, blk, 0u, stream, ga);
  else if (bkc)
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_grouped_kernel<WM, WN, false, true>, grid, blk, 0u, stream, ga);
  else
    launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_grouped_kernel<WM, WN, false, false>, grid, blk, 0u, stream, ga);
}

// One grouped launch of up to kMaxGroup problems of one operand layout.
static void gemm_group_launch(const std::vector<const Gemm*>& take, bool akc0, bool bkc0, hipStream_t stream,
                              Workspace* ws, GemmPrec prec);
// One grouped launch of up to kMaxGroup small FP64 problems.
static void gemm_small_group_launch(const std::vector<const Gemm*>& take, hipStream_t stream);

void gemm_grouped(const Gemm* qs, int count, hipStream_t stream, Workspace* ws, GemmPrec prec) {
  // Problems are sorted into the four operand layouts (which index of A and
  // of B is unit stride) and launched in groups of up to kMaxGroup per
  // layout; problems outside the 32-bit offset range or with K = 0 go
  // through gemm() one by one.
  // Small problems (register-direct kernel, any layout) form a fifth class.
  std::vector<const Gemm*> cls[5];
  for (int i = 0; i < count; ++i) {
    const Gemm& q = qs[i];
    if (q.M <= 0 || q.N <= 0 || q.batch <= 0) continue;
    const bool akc = (q.ak == 1), bkc = (q.bk == 1 && q.bn != 1);
    const bool fits = q.K > 0 && q.am >= 0 && q.ak >= 0 && q.bk >= 0 && q.bn >= 0 &&
                      (double)(q.M - 1) * q.am + (double)(q.K - 1 + BK16) * q.ak <= 536870911.0 &&
                      (double)(q.N - 1) * q.bn + (double)(q.K - 1 + BK16) * q.bk <= 536870911.0;
    if (!fits) {
      gemm(q, stream, ws, prec);
      continue;
    }
    const int l = small_gemm(q, prec) ? 4 : (akc ? 2 : 0) + (bkc ? 1 : 0);
    std::vector<const Gemm*>& c = cls[l];
    c.push_back(&q);
    if ((int)c.size() == kMaxGroup) {
      if (l == 4)
        gemm_small_group_launch(c, stream);
      else
        gemm_group_launch(c, akc, bkc, stream, ws, prec);
      c.clear();
    }
  }
  for (int l = 0; l < 4; ++l)
    if (!cls[l].empty()) gemm_group_launch(cls[l], l >= 2, l % 2 == 1, stream, ws, prec);
  if (!cls[4].empty()) gemm_small_group_launch(cls[4], stream);
}

static void gemm_small_group_launch(const std::vector<const Gemm*>& take, hipStream_t stream) {
  if (take.size() == 1) {
    gemm(*take[0], stream, nullptr, GemmPrec::F64);
    return;
  }
  GroupArgs ga{};
  ga.n = (int)take.size();
  long waves = 0;
  double flops = 0.0, bytes = 0.0;
  for (int i = 0; i < ga.n; ++i) {
    const Gemm& q = *take[i];
    KArgs& g = ga.g[i];
    g.M = q.M; g.N = q.N; g.K = q.K;
    g.A = q.A; g.am = q.am; g.ak = q.ak; g.sA = q.sA;
    g.B = q.B; g.bk = q.bk; g.bn = q.bn; g.sB = q.sB;
    g.C = q.C; g.cm = q.cm; g.cn = q.cn; g.sC = q.sC;
    g.alpha = q.alpha; g.beta = q.beta;
    g.kslices = 1;
    g.kchunk = q.K;
    g.P = nullptr;
    const int gm = (q.M + 15) / 16, gn = (q.N + 15) / 16;
    ga.gn[i] = gn;
    ga.tiles[i] = gm * gn;
    waves += (long)gm * gn * q.batch;
    if (waves > (1L << 30)) throw Error(TT_ERR_ARG, "gemm_grouped: grid too large");
    ga.end[i] = (int)waves;
    flops += 2.0 * q.M * q.N * (double)q.K * q.batch;
    bytes += 8.0 * q.batch * ((double)q.M * q.K + (double)q.K * q.N + (double)q.M * q.N * (q.beta != 0.0 ? 2 : 1));
  }
  launch_prof(PK_GEMM_F64, flops, bytes, gemm_f64_small_grouped_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256),
              0u, stream, ga);
  TT_HIP(hipGetLastError());
}

static void gemm_group_launch(const std::vector<const Gemm*>& take, bool akc0, bool bkc0, hipStream_t stream,
                              Workspace* ws, GemmPrec prec) {
  const int kstep = (prec == GemmPrec::BF16) ? BK16 : BK;
  if (take.size() == 1) {
    gemm(*take[0], stream, ws, prec);
    return;
  }
  // 64 x 64 tiles throughout (the products grouped here are small); K is
  // split where a problem's own tiles are few and its K is long, by the rule
  // of the single launch
  GroupArgs ga{};
  ga.n = (int)take.size();
  long blocks = 0, part = 0;
  double flops = 0.0, bytes = 0.0;
  int split = 0;
  for (int i = 0; i < ga.n; ++i) {
    const Gemm& q = *take[i];
    KArgs& g = ga.g[i];
    g.M = q.M; g.N = q.N; g.K = q.K;
    g.A = q.A; g.am = q.am; g.ak = q.ak; g.sA = q.sA;
    g.B = q.B; g.bk = q.bk; g.bn = q.bn; g.sB = q.sB;
    g.C = q.C; g.cm = q.cm; g.cn = q.cn; g.sC = q.sC;
    g.alpha = q.alpha; g.beta = q.beta;
    const int gm = (q.M + BM - 1) / BM, gn = (q.N + BN - 1) / BN;
    const long tiles = (long)gm * gn * q.batch;
    int ks = 1;
    if (tiles < 128 && q.K >= 16 * kstep) {
      ks = (int)std::min<long>((256 + tiles - 1) / tiles, (long)q.K / (8 * kstep));
      ks = std::max(1, std::min(ks, 64));
    }
    int chunk = (q.K + ks - 1) / ks;
    chunk = ((chunk + kstep - 1) / kstep) * kstep;
    ks = (q.K + chunk - 1) / chunk;
    g.kslices = ks;
    g.kchunk = chunk;
    g.P = nullptr;
    if (ks > 1) {
      ++split;
      part += (long)q.batch * ks * q.M * q.N;
    }
    ga.gn[i] = gn;
    ga.tiles[i] = gm * gn;
    blocks += tiles * ks;
    ga.end[i] = (int)blocks;
    flops += 2.0 * q.M * q.N * (double)q.K * q.batch;
    bytes += 8.0 * q.batch * ((double)q.M * q.K + (double)q.K * q.N + (double)q.M * q.N * (q.beta != 0.0 ? 2 : 1));
  }
  if (blocks > (1L << 30)) throw Error(TT_ERR_ARG, "gemm_grouped: grid too large");
  GroupArgs red{};
  if (split) {
    Workspace* w = ws ? ws : &g_default_ws;
    double* P0 = w->take((size_t)part);
    long off = 0, outs = 0;
    for (int i = 0; i < ga.n; ++i) {
      KArgs& g = ga.g[i];
      if (g.kslices <= 1) continue;
      const Gemm& q = *take[i];
      g.P = P0 + off;
      off += (long)q.batch * g.kslices * q.M * q.N;
      red.g[red.n] = g;
      outs += (long)q.batch * q.M * q.N;
      if (outs > (1L << 30)) throw Error(TT_ERR_ARG, "gemm_grouped: reduce too large");
      red.end[red.n] = (int)outs;
      ++red.n;
    }
  }
  if (prec == GemmPrec::BF16)
    launch_bf16_grouped<2, 2>((int)blocks, stream, ga, akc0, bkc0, flops, bytes);
  else
    launch_f64_grouped<2, 2>((int)blocks, stream, ga, akc0, bkc0, flops, bytes);
  TT_HIP(hipGetLastError());
  if (split) {
    hipLaunchKernelGGL(splitk_reduce_grouped_kernel, dim3(nblocks((long)red.end[red.n - 1], 256)), dim3(256), 0,
                       stream, red);
    TT_HIP(hipGetLastError());
  }
}

}  // namespace ttipm
