// TT algebra on the device (see tt.hpp).  Host code here only sequences kernels
// and GEMMs; every arithmetic step runs on the GPU.  The only host reads are
// the scalars that decide control flow (dot products, singular values for
// rank choices), each after a stream synchronisation.
#include "tt.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <thread>

#include "dense.hpp"
#include "ttops.hpp"

namespace ttipm {

Ctx::~Ctx() {
  if (hbuf) (void)hipHostFree(hbuf);
}

namespace {
// Idle worker contexts, each with a non-blocking stream of its own (default
// priority), kept for the life of the process.
std::mutex g_workers_mu;
std::vector<std::unique_ptr<Ctx>> g_workers;

std::unique_ptr<Ctx> acquire_worker() {
  {
    std::lock_guard<std::mutex> g(g_workers_mu);
    if (!g_workers.empty()) {
      std::unique_ptr<Ctx> w = std::move(g_workers.back());
      g_workers.pop_back();
      return w;
    }
  }
  auto w = std::make_unique<Ctx>();
  TT_HIP(hipStreamCreateWithFlags(&w->s, hipStreamNonBlocking));
  return w;
}

void release_worker(std::unique_ptr<Ctx> w) {
  std::lock_guard<std::mutex> g(g_workers_mu);
  g_workers.push_back(std::move(w));
}
}  // namespace

void run_concurrent(Ctx& c, const std::vector<std::function<void(Ctx&)>>& tasks) {
  if (tasks.empty()) return;
  if (tasks.size() == 1) {
    tasks[0](c);
    return;
  }
  c.sync();   // everything the tasks read is complete before other streams see it
  int dev = 0;
  TT_HIP(hipGetDevice(&dev));
  const size_t nw = tasks.size() - 1;
  std::vector<std::unique_ptr<Ctx>> w(nw);
  for (auto& x : w) {
    x = acquire_worker();
    x->prec = c.prec;
  }
  std::vector<std::exception_ptr> err(tasks.size());
  std::vector<std::thread> th;
  th.reserve(nw);
  for (size_t i = 0; i < nw; ++i)
    th.emplace_back([&, i] {
      pool_local_begin();
      try {
        TT_HIP(hipSetDevice(dev));
        tasks[i + 1](*w[i]);
        w[i]->sync();
      } catch (...) {
        err[i + 1] = std::current_exception();
        (void)hipStreamSynchronize(w[i]->s);
      }
      pool_local_end();
    });
  try {
    tasks[0](c);
    c.sync();
  } catch (...) {
    err[0] = std::current_exception();
  }
  for (auto& t : th) t.join();
  for (auto& x : w) release_worker(std::move(x));
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

double* Ctx::host(size_t n) {
  if (n > hbuf_n) {
    if (hbuf) (void)hipHostFree(hbuf);
    hbuf = nullptr;
    size_t want = std::max<size_t>(n, 1 << 16);
    TT_HIP(hipHostMalloc((void**)&hbuf, want * sizeof(double), hipHostMallocDefault));
    hbuf_n = want;
  }
  return hbuf;
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------
TT tt_from_host(const std::vector<std::vector<double>>& cores, const std::vector<int>& ranks, int mo, int mi,
                Ctx& c) {
  const int d = (int)cores.size();
  TT t(d, mo, mi);
  t.r = ranks;
  for (int k = 0; k < d; ++k) {
    TT_REQUIRE((long)cores[k].size() == t.core_size(k), "core size mismatch");
    t.alloc(k);
    TT_HIP(hipMemcpyAsync(t.core(k), cores[k].data(), cores[k].size() * sizeof(double), hipMemcpyHostToDevice,
                          c.s));
  }
  c.sync();
  return t;
}

TT tt_from_view(const tt_view& v, Ctx& c) {
  TT_REQUIRE(v.d >= 1 && v.ranks && v.cores, "tt_view");
  TT t(v.d, v.m_out, v.m_in);
  for (int k = 0; k <= v.d; ++k) t.r[k] = v.ranks[k];
  TT_REQUIRE(t.r[0] == 1 && t.r[v.d] == 1, "boundary ranks must be 1");
  for (int k = 0; k < v.d; ++k) {
    t.alloc(k);
    TT_HIP(hipMemcpyAsync(t.core(k), v.cores[k], t.core_size(k) * sizeof(double), hipMemcpyDeviceToDevice, c.s));
  }
  return t;
}

TT tt_clone(const TT& a, Ctx& c) {
  TT t(a.d, a.mo, a.mi);
  t.r = a.r;
  for (int k = 0; k < a.d; ++k) {
    t.alloc(k);
    TT_HIP(hipMemcpyAsync(t.core(k), a.core(k), a.core_size(k) * sizeof(double), hipMemcpyDeviceToDevice, c.s));
  }
  return t;
}

std::vector<std::vector<double>> tt_to_host(const TT& a, Ctx& c) {
  std::vector<std::vector<double>> out(a.d);
  for (int k = 0; k < a.d; ++k) {
    out[k].resize(a.core_size(k));
    TT_HIP(hipMemcpyAsync(out[k].data(), a.core(k), out[k].size() * sizeof(double), hipMemcpyDeviceToHost, c.s));
  }
  c.sync();
  return out;
}

TT tt_rank1(int d, int mo, int mi, const std::vector<double>& core, Ctx& c) {
  std::vector<std::vector<double>> cores(d, core);
  return tt_from_host(cores, std::vector<int>(d + 1, 1), mo, mi, c);
}

// ---------------------------------------------------------------------------
// algebra
// ---------------------------------------------------------------------------
TT tt_add(const std::vector<const TT*>& terms, const std::vector<double>& coef, Ctx& c) {
  TT_REQUIRE(!terms.empty() && terms.size() == coef.size(), "tt_add arguments");
  const TT& t0 = *terms[0];
  const int d = t0.d;
  const long mid = (long)t0.mo * t0.mi;
  for (auto* t : terms) TT_REQUIRE(t->d == d && t->mo == t0.mo && t->mi == t0.mi, "tt_add shapes");
  TT out(d, t0.mo, t0.mi);
  if (d == 1) {
    out.alloc(0);
    fill(out.core_size(0), 0.0, out.core(0), c.s);
    for (size_t i = 0; i < terms.size(); ++i) axpby(out.core_size(0), coef[i], terms[i]->core(0), 1.0, out.core(0), c.s);
    return out;
  }
  for (int k = 1; k < d; ++k) {
    int s = 0;
    for (auto* t : terms) s += t->r[k];
    out.r[k] = s;
  }
  for (int k = 0; k < d; ++k) {
    out.alloc(k);
    const int N0 = out.r[k], N1 = out.r[k + 1];
    if (k > 0 && k < d - 1) fill(out.core_size(k), 0.0, out.core(k), c.s);
    int o0 = 0, o1 = 0;
    for (size_t i = 0; i < terms.size(); ++i) {
      const TT& t = *terms[i];
      const int n0 = t.r[k], n1 = t.r[k + 1];
      const double a = (k == d - 1) ? coef[i] : 1.0;
      place_block(t.core(k), n0, mid, n1, out.core(k), N0, N1, (k == 0) ? 0 : o0, (k == d - 1) ? 0 : o1, a, c.s);
      o0 += n0;
      o1 += n1;
    }
  }
  return out;
}

void tt_scale(TT& a, double s, Ctx& c) { axpby(a.core_size(a.d - 1), 0.0, a.core(a.d - 1), s, a.core(a.d - 1), c.s); }

TT tt_kron(const TT& A, const TT& B, Ctx& c) {
  TT_REQUIRE(A.d == B.d, "kron d");
  TT out(A.d, A.mo * B.mo, A.mi * B.mi);
  for (int k = 0; k <= A.d; ++k) out.r[k] = A.r[k] * B.r[k];
  for (int k = 0; k < A.d; ++k) {
    out.alloc(k);
    kron_core(A.core(k), A.r[k], A.mo, A.mi, A.r[k + 1], B.core(k), B.r[k], B.mo, B.mi, B.r[k + 1], out.core(k), c.s);
  }
  return out;
}

TT tt_diag(const TT& v, Ctx& c) {
  TT_REQUIRE(v.mi == 1, "diag of a vector");
  TT out(v.d, v.mo, v.mo);
  out.r = v.r;
  for (int k = 0; k < v.d; ++k) {
    out.alloc(k);
    diag_core(v.core(k), v.r[k], v.mo, v.r[k + 1], out.core(k), c.s);
  }
  return out;
}

TT tt_matvec(const TT& A, const TT& x, Ctx& c) {
  TT_REQUIRE(A.d == x.d && A.mi == x.mo && x.mi == 1, "matvec shapes");
  TT out(A.d, A.mo, 1);
  for (int k = 0; k <= A.d; ++k) out.r[k] = A.r[k] * x.r[k];
  for (int k = 0; k < A.d; ++k) {
    out.alloc(k);
    matvec_core(A.core(k), A.r[k], A.mo, A.mi, A.r[k + 1], x.core(k), x.r[k], x.r[k + 1], out.core(k), c.s);
  }
  return out;
}

TT tt_matmat(const TT& A, const TT& B, Ctx& c) {
  TT_REQUIRE(A.d == B.d && A.mi == B.mo, "matmat shapes");
  TT out(A.d, A.mo, B.mi);
  for (int k = 0; k <= A.d; ++k) out.r[k] = A.r[k] * B.r[k];
  for (int k = 0; k < A.d; ++k) {
    out.alloc(k);
    matmat_core(A.core(k), A.r[k], A.mo, A.mi, A.r[k + 1], B.core(k), B.r[k], B.mi, B.r[k + 1], out.core(k), c.s);
  }
  return out;
}

TT tt_as_matrix(const TT& v, int n, Ctx& c) {
  TT_REQUIRE(v.mi == 1 && v.mo == n * n, "as_matrix");
  TT t = tt_clone(v, c);
  t.mo = n;
  t.mi = n;
  return t;
}

TT tt_as_vector(const TT& m, Ctx& c) {
  TT t = tt_clone(m, c);
  t.mo = m.mo * m.mi;
  t.mi = 1;
  return t;
}

TT tt_transpose(const TT& A, Ctx& c) {
  TT out(A.d, A.mi, A.mo);
  out.r = A.r;
  for (int k = 0; k < A.d; ++k) {
    out.alloc(k);
    permute(A.core(k), out.core(k), {A.r[k], A.mo, A.mi, A.r[k + 1]}, {0, 2, 1, 3}, c.s);
  }
  return out;
}

// <x, y> by left-to-right identity environments.
double tt_dot(const TT& x, const TT& y, Ctx& c) {
  TT_REQUIRE(x.d == y.d && x.mo * x.mi == y.mo * y.mi, "dot shapes");
  const int m = x.mo * x.mi;
  int maxr = 1;
  for (int k = 0; k <= x.d; ++k) maxr = std::max(maxr, x.r[k] * y.r[k]);
  DevBuf e0(maxr), e1(maxr);
  fill(1, 1.0, e0.get(), c.s);
  for (int k = 0; k < x.d; ++k) {
    env_left_step(e0.get(), x.r[k], 1, y.r[k], x.core(k), m, x.r[k + 1], nullptr, 1, m, y.core(k), y.r[k + 1],
                  e1.get(), c);
    std::swap(e0, e1);
  }
  double* h = c.host(1);
  TT_HIP(hipMemcpyAsync(h, e0.get(), sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return h[0];
}

double tt_norm(const TT& x, Ctx& c) {
  double v = tt_dot(x, x, c);
  return v > 0 ? std::sqrt(v) : 0.0;
}

double tt_sandwich(const TT& u, const TT& A, const TT& v, Ctx& c) {
  TT_REQUIRE(u.d == A.d && v.d == A.d && u.mo == A.mo && v.mo == A.mi, "sandwich shapes");
  int maxr = 1;
  for (int k = 0; k <= u.d; ++k) maxr = std::max(maxr, u.r[k] * A.r[k] * v.r[k]);
  DevBuf e0(maxr), e1(maxr);
  fill(1, 1.0, e0.get(), c.s);
  for (int k = 0; k < u.d; ++k) {
    env_left_step(e0.get(), u.r[k], A.r[k], v.r[k], u.core(k), A.mo, u.r[k + 1], A.core(k), A.r[k + 1], A.mi,
                  v.core(k), v.r[k + 1], e1.get(), c);
    std::swap(e0, e1);
  }
  double* h = c.host(1);
  TT_HIP(hipMemcpyAsync(h, e0.get(), sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return h[0];
}

// <Oi vi, Oj vj> by a left-to-right sweep over a four-layer environment
// E[a][alpha][beta][c] (a, c: ranks of vi, vj; alpha, beta: ranks of Oi, Oj),
// four GEMM stages per core: vj, then Oj over its input mode, then Oi over the
// shared output mode, then vi over Oi's input mode.
namespace {
// gathers the scalars at the given device addresses into out[0..n)
constexpr int kGather = 64;
struct GatherArgs {
  const double* p[kGather];
  int n;
};
__global__ void gather_scalars_kernel(GatherArgs g, double* out) {
  const int t = threadIdx.x;
  if (t < g.n) out[t] = *g.p[t];
}
}  // namespace

std::vector<double> tt_op_dots(const std::vector<OpDotPair>& pairs, Ctx& c) {
  const int np = (int)pairs.size();
  std::vector<double> out(np, 0.0);
  if (np == 0) return out;
  const TT& v0 = *pairs[0].vi;
  const int d = v0.d, m = v0.mo;
  for (const OpDotPair& q : pairs) {
    TT_REQUIRE(q.vi->d == d && q.vj->d == d && q.vi->mo == m && q.vj->mo == m && q.vi->mi == 1 && q.vj->mi == 1,
               "op_dot vector shapes");
    for (const TT* O : {q.Oi, q.Oj})
      if (O) TT_REQUIRE(O->d == d && O->mo == m && O->mi == m, "op_dot operator shapes");
  }
  std::vector<double> eye((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) eye[(size_t)i * m + i] = 1.0;
  TT Id = tt_rank1(d, m, m, eye, c);
  std::vector<const TT*> A(np), B(np);
  for (int p = 0; p < np; ++p) {
    A[p] = pairs[p].Oi ? pairs[p].Oi : &Id;
    B[p] = pairs[p].Oj ? pairs[p].Oj : &Id;
  }
  // per pair: environments e0, e1 and stage buffers t1, t2, carved from one slab
  std::vector<size_t> emax(np, 1), tmax(np, 1);
  size_t total = 0;
  for (int p = 0; p < np; ++p) {
    const TT &vi = *pairs[p].vi, &vj = *pairs[p].vj, &a = *A[p], &bb = *B[p];
    for (int k = 0; k <= d; ++k) emax[p] = std::max(emax[p], (size_t)vi.r[k] * a.r[k] * bb.r[k] * vj.r[k]);
    for (int k = 0; k < d; ++k) {
      const size_t ra = vi.r[k], al = a.r[k], be = bb.r[k];
      const size_t a2 = vi.r[k + 1], al2 = a.r[k + 1], be2 = bb.r[k + 1], c2 = vj.r[k + 1];
      tmax[p] = std::max({tmax[p], ra * al * be * m * c2, ra * al * c2 * m * be2, ra * c2 * be2 * m * al2});
    }
    total += 2 * ((emax[p] + 31) & ~size_t(31)) + 2 * ((tmax[p] + 31) & ~size_t(31));
  }
  // the permuted core of each distinct right operator, per core
  std::vector<const TT*> ops;
  std::vector<int> op_of(np);
  for (int p = 0; p < np; ++p) {
    int f = -1;
    for (int i = 0; i < (int)ops.size(); ++i)
      if (ops[i] == B[p]) f = i;
    if (f < 0) {
      f = (int)ops.size();
      ops.push_back(B[p]);
    }
    op_of[p] = f;
  }
  std::vector<size_t> pmax(ops.size());
  for (size_t i = 0; i < ops.size(); ++i) {
    pmax[i] = (size_t)ops[i]->max_rank() * ops[i]->max_rank() * m * m;
    total += (pmax[i] + 31) & ~size_t(31);
  }
  DevBuf slab(total), res(np);
  std::vector<double*> e0(np), e1(np), t1(np), t2(np), pB(ops.size());
  {
    double* q = slab.get();
    auto take = [&](size_t n) {
      double* r = q;
      q += (n + 31) & ~size_t(31);
      return r;
    };
    for (int p = 0; p < np; ++p) {
      e0[p] = take(emax[p]);
      e1[p] = take(emax[p]);
      t1[p] = take(tmax[p]);
      t2[p] = take(tmax[p]);
    }
    for (size_t i = 0; i < ops.size(); ++i) pB[i] = take(pmax[i]);
  }
  for (int p = 0; p < np; ++p) fill(1, 1.0, e0[p], c.s);
  std::vector<Gemm> g(np);
  std::vector<PermJob> pj;
  for (int k = 0; k < d; ++k) {
    // Oj [be][i][j][be2] -> [(be,j)][(i,be2)], once per distinct operator
    pj.clear();
    for (size_t i = 0; i < ops.size(); ++i)
      pj.push_back({ops[i]->core(k), pB[i], {ops[i]->r[k], m, m, ops[i]->r[k + 1]}, {0, 2, 1, 3}});
    permute_many(pj, c.s);
    // T1[(a,al,be)][(j,c2)] = E[(a,al,be)][c] vj[c][(j,c2)]
    for (int p = 0; p < np; ++p) {
      const TT &vi = *pairs[p].vi, &vj = *pairs[p].vj;
      const int a = vi.r[k], al = A[p]->r[k], be = B[p]->r[k], cc = vj.r[k], c2 = vj.r[k + 1];
      g[p] = gemm_nn(a * al * be, m * c2, cc, e0[p], cc, vj.core(k), (long)m * c2, t1[p], (long)m * c2);
    }
    gemm_grouped(g.data(), np, c.s, &c.ws, GemmPrec::F64);
    // [a][al][be][j][c2] -> [a][al][c2][be][j]
    pj.clear();
    for (int p = 0; p < np; ++p) {
      const int a = pairs[p].vi->r[k], al = A[p]->r[k], be = B[p]->r[k], c2 = pairs[p].vj->r[k + 1];
      pj.push_back({t1[p], t2[p], {a, al, be, m, c2}, {0, 1, 4, 2, 3}});
    }
    permute_many(pj, c.s);
    // T2[(a,al,c2)][(i,be2)] = T1'[(a,al,c2)][(be,j)] Oj'[(be,j)][(i,be2)]
    for (int p = 0; p < np; ++p) {
      const int a = pairs[p].vi->r[k], al = A[p]->r[k], be = B[p]->r[k], c2 = pairs[p].vj->r[k + 1];
      const int be2 = B[p]->r[k + 1];
      g[p] = gemm_nn(a * al * c2, m * be2, be * m, t2[p], (long)be * m, pB[op_of[p]], (long)m * be2, t1[p],
                     (long)m * be2);
    }
    gemm_grouped(g.data(), np, c.s, &c.ws, GemmPrec::F64);
    // [a][al][c2][i][be2] -> [a][c2][be2][al][i]
    pj.clear();
    for (int p = 0; p < np; ++p) {
      const int a = pairs[p].vi->r[k], al = A[p]->r[k], c2 = pairs[p].vj->r[k + 1], be2 = B[p]->r[k + 1];
      pj.push_back({t1[p], t2[p], {a, al, c2, m, be2}, {0, 2, 4, 1, 3}});
    }
    permute_many(pj, c.s);
    // T3[(a,c2,be2)][(j,al2)] = T2'[(a,c2,be2)][(al,i)] Oi[(al,i)][(j,al2)]
    for (int p = 0; p < np; ++p) {
      const int a = pairs[p].vi->r[k], al = A[p]->r[k], c2 = pairs[p].vj->r[k + 1], be2 = B[p]->r[k + 1];
      const int al2 = A[p]->r[k + 1];
      g[p] = gemm_nn(a * c2 * be2, m * al2, al * m, t2[p], (long)al * m, A[p]->core(k), (long)m * al2, t1[p],
                     (long)m * al2);
    }
    gemm_grouped(g.data(), np, c.s, &c.ws, GemmPrec::F64);
    // [a][c2][be2][j][al2] -> [a][j][al2][be2][c2]
    pj.clear();
    for (int p = 0; p < np; ++p) {
      const int a = pairs[p].vi->r[k], c2 = pairs[p].vj->r[k + 1], be2 = B[p]->r[k + 1], al2 = A[p]->r[k + 1];
      pj.push_back({t1[p], t2[p], {a, c2, be2, m, al2}, {0, 3, 4, 2, 1}});
    }
    permute_many(pj, c.s);
    // E'[a2][(al2,be2,c2)] = sum_(a,j) vi[(a,j)][a2] T3'[(a,j)][(al2,be2,c2)]
    for (int p = 0; p < np; ++p) {
      const TT& vi = *pairs[p].vi;
      const int a = vi.r[k], a2 = vi.r[k + 1], al2 = A[p]->r[k + 1], be2 = B[p]->r[k + 1];
      const int c2 = pairs[p].vj->r[k + 1];
      Gemm q;
      q.M = a2; q.N = al2 * be2 * c2; q.K = a * m;
      q.A = vi.core(k); q.am = 1; q.ak = a2;
      q.B = t2[p]; q.bk = (long)al2 * be2 * c2; q.bn = 1;
      q.C = e1[p]; q.cm = (long)al2 * be2 * c2; q.cn = 1;
      g[p] = q;
    }
    gemm_grouped(g.data(), np, c.s, &c.ws, GemmPrec::F64);
    std::swap(e0, e1);
  }
  for (int p0 = 0; p0 < np; p0 += kGather) {
    GatherArgs ga{};
    ga.n = std::min(kGather, np - p0);
    for (int i = 0; i < ga.n; ++i) ga.p[i] = e0[p0 + i];
    hipLaunchKernelGGL(gather_scalars_kernel, dim3(1), dim3(kGather), 0, c.s, ga, res.get() + p0);
    TT_HIP(hipGetLastError());
  }
  double* h = c.host(np);
  TT_HIP(hipMemcpyAsync(h, res.get(), sizeof(double) * np, hipMemcpyDeviceToHost, c.s));
  c.sync();
  for (int p = 0; p < np; ++p) out[p] = h[p];
  return out;
}

double tt_op_dot(const TT& vi, const TT* Oi, const TT& vj, const TT* Oj, Ctx& c) {
  return tt_op_dots({OpDotPair{&vi, Oi, &vj, Oj}}, c)[0];
}

// ---------------------------------------------------------------------------
// environments and local products: three GEMM stages each
// ---------------------------------------------------------------------------
void permute_op_core(const double* O, int R, int m, int Rp, double* out, hipStream_t s) {
  // [alpha][i][j][beta] -> [i][beta][alpha][j]
  permute(O, out, {R, m, m, Rp}, {1, 3, 0, 2}, s);
}

namespace {

// The GEMMs of one environment step, in order, with the scratch they use; the
// left step with an operator permutes the operator core before its second GEMM.
struct EnvPlan {
  Gemm g[3];
  int ng = 0;
  bool permute_core = false;   // permute O into perm before g[1]
  const double* O = nullptr;
  int R = 0, mo = 0, mi = 0, Rp = 0;
  double* perm = nullptr;
};

EnvPlan plan_left(const double* phi, int ra, int R, int rc, const double* V, int mo, int ra2, const double* O,
                  int Rp, int mi, const double* U, int rc2, double* out, double* t1, double* t2, double* perm) {
  EnvPlan P;
  if (O == nullptr) {
    TT_REQUIRE(R == 1 && Rp == 1 && mo == mi, "identity environment shapes");
    // t1[a][(i,c2)] = phi[a][c] U[c][(i,c2)];  out[a2][c2] = sum_(a,i) V[(a,i)][a2] t1[(a,i)][c2]
    P.g[0] = gemm_nn(ra, mi * rc2, rc, phi, rc, U, mi * rc2, t1, mi * rc2);
    Gemm& g = P.g[1];
    g.M = ra2; g.N = rc2; g.K = ra * mo;
    g.A = V; g.am = 1; g.ak = ra2;
    g.B = t1; g.bk = rc2; g.bn = 1;
    g.C = out; g.cm = rc2; g.cn = 1;
    P.ng = 2;
    return P;
  }
  // stage 1: t1[(a,alpha)][(j,c2)] = phi[(a,alpha)][c] U[c][(j,c2)]
  P.g[0] = gemm_nn(ra * R, mi * rc2, rc, phi, rc, U, mi * rc2, t1, mi * rc2);
  // stage 2: t2[a][(i,beta)][c2] = O'[(i,beta)][(alpha,j)] t1[a][(alpha,j)][c2]
  P.permute_core = true;
  P.O = O; P.R = R; P.mo = mo; P.mi = mi; P.Rp = Rp; P.perm = perm;
  {
    Gemm& g = P.g[1];
    g.M = mo * Rp; g.N = rc2; g.K = R * mi; g.batch = ra;
    g.A = perm; g.am = R * mi; g.ak = 1; g.sA = 0;
    g.B = t1; g.bk = rc2; g.bn = 1; g.sB = (long)R * mi * rc2;
    g.C = t2; g.cm = rc2; g.cn = 1; g.sC = (long)mo * Rp * rc2;
  }
  // stage 3: out[a2][(beta,c2)] = sum_(a,i) V[(a,i)][a2] t2[(a,i)][(beta,c2)]
  {
    Gemm& g = P.g[2];
    g.M = ra2; g.N = Rp * rc2; g.K = ra * mo;
    g.A = V; g.am = 1; g.ak = ra2;
    g.B = t2; g.bk = (long)Rp * rc2; g.bn = 1;
    g.C = out; g.cm = (long)Rp * rc2; g.cn = 1;
  }
  P.ng = 3;
  return P;
}

EnvPlan plan_right(const double* phi, int ra2, int Rp, int rc2, const double* V, int mo, int ra, const double* O,
                   int R, int mi, const double* U, int rc, double* out, double* t1, double* t2) {
  EnvPlan P;
  if (O == nullptr) {
    TT_REQUIRE(R == 1 && Rp == 1 && mo == mi, "identity environment shapes");
    // t1[(c,i)][a2] = sum_c2 U[(c,i)][c2] phi[a2][c2]
    Gemm& g1 = P.g[0];
    g1.M = rc * mi; g1.N = ra2; g1.K = rc2;
    g1.A = U; g1.am = rc2; g1.ak = 1;
    g1.B = phi; g1.bk = 1; g1.bn = rc2;
    g1.C = t1; g1.cm = ra2; g1.cn = 1;
    // out[a][c] = sum_(i,a2) V[a][(i,a2)] t1[c][(i,a2)]
    Gemm& g2 = P.g[1];
    g2.M = ra; g2.N = rc; g2.K = mo * ra2;
    g2.A = V; g2.am = (long)mo * ra2; g2.ak = 1;
    g2.B = t1; g2.bk = 1; g2.bn = (long)mi * ra2;
    g2.C = out; g2.cm = rc; g2.cn = 1;
    P.ng = 2;
    return P;
  }
  // stage 1 (batched over a2): t1[a2][(c,j)][beta] = sum_c2 U[(c,j)][c2] phi[a2][beta][c2]
  {
    Gemm& g = P.g[0];
    g.M = rc * mi; g.N = Rp; g.K = rc2; g.batch = ra2;
    g.A = U; g.am = rc2; g.ak = 1; g.sA = 0;
    g.B = phi; g.bk = 1; g.bn = rc2; g.sB = (long)Rp * rc2;
    g.C = t1; g.cm = Rp; g.cn = 1; g.sC = (long)rc * mi * Rp;
  }
  // stage 2: t2[(alpha,i)][(a2,c)] = sum_(j,beta) O[(alpha,i)][(j,beta)] t1[(a2,c)][(j,beta)]
  {
    Gemm& g = P.g[1];
    g.M = R * mo; g.N = ra2 * rc; g.K = mi * Rp;
    g.A = O; g.am = (long)mi * Rp; g.ak = 1;
    g.B = t1; g.bk = 1; g.bn = (long)mi * Rp;
    g.C = t2; g.cm = (long)ra2 * rc; g.cn = 1;
  }
  // stage 3 (batched over alpha): out[a][alpha][c] = sum_(i,a2) V[a][(i,a2)] t2[alpha][(i,a2)][c]
  {
    Gemm& g = P.g[2];
    g.M = ra; g.N = rc; g.K = mo * ra2; g.batch = R;
    g.A = V; g.am = (long)mo * ra2; g.ak = 1; g.sA = 0;
    g.B = t2; g.bk = rc; g.bn = 1; g.sB = (long)mo * ra2 * rc;
    g.C = out; g.cm = (long)R * rc; g.cn = 1; g.sC = rc;
  }
  P.ng = 3;
  return P;
}

// The plans' GEMMs level by level: the k-th GEMMs of all plans are independent
// (each plan owns its scratch and output), so each level is grouped launches.
void run_plans(std::vector<EnvPlan>& plans, Ctx& c) {
  for (int lv = 0; lv < 3; ++lv) {
    std::vector<Gemm> gs;
    std::vector<PermJob> jobs;   // operator cores the second GEMMs read permuted, in one launch
    for (EnvPlan& P : plans) {
      if (lv >= P.ng) continue;
      if (lv == 1 && P.permute_core) jobs.push_back({P.O, P.perm, {P.R, P.mo, P.mi, P.Rp}, {1, 3, 0, 2}});
      gs.push_back(P.g[lv]);
    }
    if (!jobs.empty()) permute_many(jobs, c.s);
    if (!gs.empty()) gemm_grouped(gs.data(), (int)gs.size(), c.s, &c.ws, c.prec);
  }
}

}  // namespace

void env_left_step(const double* phi, int ra, int R, int rc, const double* V, int mo, int ra2, const double* O,
                   int Rp, int mi, const double* U, int rc2, double* out, Ctx& c) {
  c.t1.reserve((size_t)ra * R * mi * rc2);
  if (O) {
    c.perm.reserve((size_t)R * mo * mi * Rp);
    c.t2.reserve((size_t)ra * mo * Rp * rc2);
  }
  std::vector<EnvPlan> plans{plan_left(phi, ra, R, rc, V, mo, ra2, O, Rp, mi, U, rc2, out, c.t1.get(), c.t2.get(),
                                       c.perm.get())};
  run_plans(plans, c);
}

void env_right_step(const double* phi, int ra2, int Rp, int rc2, const double* V, int mo, int ra,
                    const double* O, int R, int mi, const double* U, int rc, double* out, Ctx& c) {
  c.t1.reserve((size_t)ra2 * rc * mi * Rp);
  if (O) c.t2.reserve((size_t)R * mo * ra2 * rc);
  std::vector<EnvPlan> plans{plan_right(phi, ra2, Rp, rc2, V, mo, ra, O, R, mi, U, rc, out, c.t1.get(), c.t2.get())};
  run_plans(plans, c);
}

void env_steps(const std::vector<EnvStepArgs>& steps, bool left, Ctx& c) {
  std::vector<EnvPlan> plans;
  plans.reserve(steps.size());
  size_t nb = 0;
  auto buf = [&](size_t n) {
    if (c.gbuf.size() <= nb) c.gbuf.resize(nb + 1);
    c.gbuf[nb].reserve(n);
    return c.gbuf[nb++].get();
  };
  for (const EnvStepArgs& a : steps) {
    if (left) {
      double* t1 = buf((size_t)a.ra * a.R * a.mi * a.rc2);
      double* t2 = a.O ? buf((size_t)a.ra * a.mo * a.Rp * a.rc2) : nullptr;
      double* perm = a.O ? buf((size_t)a.R * a.mo * a.mi * a.Rp) : nullptr;
      plans.push_back(plan_left(a.phi, a.ra, a.R, a.rc, a.V, a.mo, a.ra2, a.O, a.Rp, a.mi, a.U, a.rc2, a.out, t1, t2,
                                perm));
    } else {
      // the fields hold env_right_step's arguments in its order:
      // (phi, ra2, Rp, rc2, V, mo, ra, O, R, mi, U, rc, out)
      const int ra2 = a.ra, Rp = a.R, rc2 = a.rc, ra = a.ra2, R = a.Rp, rc = a.rc2;
      double* t1 = buf((size_t)ra2 * rc * a.mi * Rp);
      double* t2 = a.O ? buf((size_t)R * a.mo * ra2 * rc) : nullptr;
      plans.push_back(plan_right(a.phi, ra2, Rp, rc2, a.V, a.mo, ra, a.O, R, a.mi, a.U, rc, a.out, t1, t2));
    }
  }
  run_plans(plans, c);
}

void local_apply(const double* phiL, int r, int R, int rc, const double* Operm, int m, const double* phiR, int s,
                 int Rp, int rd, const double* x, double* y, double alpha, double beta, Ctx& c) {
  // y[a][i][b] = alpha sum phiL[a][al][c] O[al][i][j][be] x[c][j][e] phiR[b][be][e] + beta y
  if (Operm == nullptr) {
    TT_REQUIRE(R == 1 && Rp == 1, "identity local operator");
    c.t1.reserve((size_t)r * m * rd);
    gemm(gemm_nn(r, m * rd, rc, phiL, rc, x, m * rd, c.t1.get(), m * rd), c.s, &c.ws, c.prec);
    Gemm g;
    g.M = r * m; g.N = s; g.K = rd;
    g.A = c.t1.get(); g.am = rd; g.ak = 1;
    g.B = phiR; g.bk = 1; g.bn = rd;
    g.C = y; g.cm = s; g.cn = 1;
    g.alpha = alpha; g.beta = beta;
    gemm(g, c.s, &c.ws, c.prec);
    return;
  }
  // stage 1: t1[(a,alpha)][(j,e)] = phiL[(a,alpha)][c] x[c][(j,e)]
  c.t1.reserve((size_t)r * R * m * rd);
  gemm(gemm_nn(r * R, m * rd, rc, phiL, rc, x, m * rd, c.t1.get(), m * rd), c.s, &c.ws, c.prec);
  // stage 2 (batched over a): t2[a][(i,beta)][e] = O'[(i,beta)][(alpha,j)] t1[a][(alpha,j)][e]
  c.t2.reserve((size_t)r * m * Rp * rd);
  {
    Gemm g;
    g.M = m * Rp; g.N = rd; g.K = R * m; g.batch = r;
    g.A = Operm; g.am = (long)R * m; g.ak = 1; g.sA = 0;
    g.B = c.t1.get(); g.bk = rd; g.bn = 1; g.sB = (long)R * m * rd;
    g.C = c.t2.get(); g.cm = rd; g.cn = 1; g.sC = (long)m * Rp * rd;
    gemm(g, c.s, &c.ws, c.prec);
  }
  // stage 3: y[(a,i)][b] = alpha sum_(beta,e) t2[(a,i)][(beta,e)] phiR[b][(beta,e)] + beta y
  {
    Gemm g;
    g.M = r * m; g.N = s; g.K = Rp * rd;
    g.A = c.t2.get(); g.am = (long)Rp * rd; g.ak = 1;
    g.B = phiR; g.bk = 1; g.bn = (long)Rp * rd;
    g.C = y; g.cm = s; g.cn = 1;
    g.alpha = alpha; g.beta = beta;
    gemm(g, c.s, &c.ws, c.prec);
  }
}

void local_apply_many(const std::vector<LocalApplyArgs>& v, Ctx& c, Arena* arena, bool dry, size_t* ws_need) {
  if (v.empty()) return;
  size_t nb = 0;
  auto buf = [&](size_t n) {
    if (arena) return arena->take(n);
    if (c.gbuf.size() <= nb) c.gbuf.resize(nb + 1);
    c.gbuf[nb].reserve(n);
    return c.gbuf[nb++].get();
  };
  std::vector<Gemm> g1, g2, g3;
  for (const LocalApplyArgs& a : v) {
    double* t1 = buf((size_t)a.r * a.R * a.m * a.rd);
    // stage 1: t1[(a,alpha)][(j,e)] = phiL[(a,alpha)][c] x[c][(j,e)]
    g1.push_back(gemm_nn(a.r * a.R, a.m * a.rd, a.rc, a.phiL, a.rc, a.x, (long)a.m * a.rd, t1, (long)a.m * a.rd));
    const double* last = t1;
    if (a.Operm) {
      // stage 2 (batched over a): t2[a][(i,beta)][e] = O'[(i,beta)][(alpha,j)] t1[a][(alpha,j)][e]
      double* t2 = buf((size_t)a.r * a.m * a.Rp * a.rd);
      Gemm g;
      g.M = a.m * a.Rp; g.N = a.rd; g.K = a.R * a.m; g.batch = a.r;
      g.A = a.Operm; g.am = (long)a.R * a.m; g.ak = 1; g.sA = 0;
      g.B = t1; g.bk = a.rd; g.bn = 1; g.sB = (long)a.R * a.m * a.rd;
      g.C = t2; g.cm = a.rd; g.cn = 1; g.sC = (long)a.m * a.Rp * a.rd;
      g2.push_back(g);
      last = t2;
    } else {
      TT_REQUIRE(a.R == 1 && a.Rp == 1, "identity local operator");
    }
    // stage 3: y[(a,i)][b] = alpha sum_(beta,e) t2[(a,i)][(beta,e)] phiR[b][(beta,e)] + beta y
    Gemm g;
    g.M = a.r * a.m; g.N = a.s; g.K = a.Rp * a.rd;
    g.A = last; g.am = (long)a.Rp * a.rd; g.ak = 1;
    g.B = a.phiR; g.bk = 1; g.bn = (long)a.Rp * a.rd;
    g.C = a.y; g.cm = a.s; g.cn = 1;
    g.alpha = a.alpha; g.beta = a.beta;
    g3.push_back(g);
  }
  // last stages in list order, a launch cut wherever an output repeats
  std::vector<std::pair<size_t, size_t>> cuts;
  {
    size_t b = 0;
    for (size_t e = 0; e <= g3.size(); ++e) {
      bool cut = e == g3.size();
      for (size_t q = b; q < e && !cut; ++q) cut = g3[q].C == g3[e].C;
      if (cut && e > b) {
        cuts.push_back({b, e});
        b = e;
      }
    }
  }
  if (dry) {
    // every grouped call reuses the partials region from its start
    auto need = [&](const Gemm* q, size_t n) {
      size_t t = 0;
      for (size_t i = 0; i < n; ++i) t += gemm_splitk_need(q[i], c.prec);
      return t;
    };
    size_t w = std::max(need(g1.data(), g1.size()), need(g2.data(), g2.size()));
    for (const auto& ct : cuts) w = std::max(w, need(g3.data() + ct.first, ct.second - ct.first));
    if (ws_need) *ws_need = std::max(*ws_need, w);
    return;
  }
  Workspace fixed_ws;
  Workspace* ws = &c.ws;
  if (arena) {
    double* rest = arena->take(0);
    fixed_ws.fixed = rest;
    fixed_ws.fixed_n = arena->cap > arena->used ? arena->cap - arena->used : 0;
    ws = &fixed_ws;
  }
  gemm_grouped(g1.data(), (int)g1.size(), c.s, ws, c.prec);
  gemm_grouped(g2.data(), (int)g2.size(), c.s, ws, c.prec);
  for (const auto& ct : cuts) gemm_grouped(g3.data() + ct.first, (int)(ct.second - ct.first), c.s, ws, c.prec);
}

// ---------------------------------------------------------------------------
// SVD and orthogonalisation
// ---------------------------------------------------------------------------
__global__ void upper_to_rowmajor_kernel(const double* Acm, int lda, int k, int n, double* R) {
  // R (k x n row-major) = upper triangle of the column-major QR output
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)k * n) return;
  int i = (int)(t / n), j = (int)(t % n);
  R[t] = (i <= j) ? Acm[(long)j * lda + i] : 0.0;
}

// Householder QR of a row-major matrix given as its column-major transpose:
// the input `Mt_cm` is column-major (m x n) = row-major (n x m).  Returns Q
// column-major (m x k) and R row-major (k x n), k = min(m, n).
static void qr_colmajor(double* A, int m, int n, double* Q, double* R, Ctx& c) {
  const int k = std::min(m, n);
  c.dscr3.reserve((size_t)k + 1);
  dense_qr(A, m, n, m, c.dscr3.get(), c.s);
  hipLaunchKernelGGL(upper_to_rowmajor_kernel, dim3(nblocks((long)k * n, 256)), dim3(256), 0, c.s, A, m, k, n, R);
  TT_HIP(hipGetLastError());
  dense_qr_form_q(A, m, n, m, c.dscr3.get(), Q, k, m, c.s);
}

void svd_rowmajor(const double* M, int rows, int cols, SvdOut& out, Ctx& c) {
  // Jacobi works on the columns of a column-major matrix.  For rows >= cols we
  // factor M (column-major copy = transpose of the row-major data); otherwise
  // M^T, whose column-major form is the row-major M itself.
  const bool tall = rows >= cols;
  const int m = tall ? rows : cols;     // length of the Jacobi columns
  const int n = tall ? cols : rows;     // number of Jacobi columns
  const int k = n;
  out.k = k;
  DevBuf A((size_t)m * n);
  if (tall)
    permute(M, A.get(), {rows, cols}, {1, 0}, c.s);
  else
    TT_HIP(hipMemcpyAsync(A.get(), M, sizeof(double) * (size_t)m * n, hipMemcpyDeviceToDevice, c.s));
  DevBuf Ucm((size_t)m * n), Vcm((size_t)n * n), sig(n), work((size_t)n * n);
  c.ired.reserve((size_t)n + 8);
  int* iw = reinterpret_cast<int*>(c.ired.get());
  if (m > 2 * n || (!dense_svd_fits_lds(m, n) && dense_svd_fits_lds(n, n))) {
    // QR first: A = Q R with R (n x n); SVD of R keeps the Jacobi sweeps on
    // n x n -- for tall matrices, and wherever that lets the sweeps run with
    // both R and the rotations resident in LDS.
    DevBuf Q((size_t)m * n), R((size_t)n * n), Rcm((size_t)n * n), Ur((size_t)n * n);
    qr_colmajor(A.get(), m, n, Q.get(), R.get(), c);
    permute(R.get(), Rcm.get(), {n, n}, {1, 0}, c.s);
    dense_svd(Rcm.get(), n, n, Ur.get(), sig.get(), Vcm.get(), work.get(), iw, c.s);
    // Ucm (m x n col-major) = Q Ur : row-major view Ucm^T (n x m) = Ur^T Q^T
    Gemm g;
    g.M = n; g.N = m; g.K = n;
    g.A = Ur.get(); g.am = n; g.ak = 1;          // Ur^T[c][j] = Ur(j,c) = Ur[c*n + j]
    g.B = Q.get(); g.bk = m; g.bn = 1;           // Q^T[j][i] = Q(i,j) = Q[j*m + i]
    g.C = Ucm.get(); g.cm = m; g.cn = 1;
    gemm(g, c.s, &c.ws, GemmPrec::F64);
  } else {
    dense_svd(A.get(), m, n, Ucm.get(), sig.get(), Vcm.get(), work.get(), iw, c.s);
  }
  out.sigma.resize(k);
  TT_HIP(hipMemcpyAsync(out.sigma.data(), sig.get(), sizeof(double) * k, hipMemcpyDeviceToHost, c.s));
  out.U.reserve((size_t)rows * k);
  out.Vt.reserve((size_t)k * cols);
  if (tall) {
    // U row-major (rows x k) = transpose of Ucm; Vt row-major (k x cols) = Vcm buffer
    permute(Ucm.get(), out.U.get(), {k, rows}, {1, 0}, c.s);
    TT_HIP(hipMemcpyAsync(out.Vt.get(), Vcm.get(), sizeof(double) * (size_t)k * cols, hipMemcpyDeviceToDevice, c.s));
  } else {
    // M^T = U' S V'^T: U (rows x k) = V' -> transpose of Vcm; Vt (k x cols) = U'^T = Ucm buffer
    permute(Vcm.get(), out.U.get(), {k, rows}, {1, 0}, c.s);
    TT_HIP(hipMemcpyAsync(out.Vt.get(), Ucm.get(), sizeof(double) * (size_t)k * cols, hipMemcpyDeviceToDevice, c.s));
  }
  c.sync();
}

void svd_rowmajor_side(const double* M, int rows, int cols, bool left, SvdOut& out, Ctx& c) {
  // T is the matrix whose left singular vectors are wanted: M itself (left) or
  // M^T (right, whose left vectors are the right vectors of M).  The Jacobi
  // sweeps then need no rotation accumulator: the vectors are the normalised
  // final columns.
  const int mt = left ? rows : cols, nt = left ? cols : rows;
  const int k = std::min(mt, nt);
  out.k = k;
  DevBuf Ut((size_t)mt * k), sig(k);
  c.ired.reserve((size_t)k + 8);
  int* iw = reinterpret_cast<int*>(c.ired.get());
  if (mt >= nt) {
    // column-major T: M^T's is the row-major M itself, M's is its transpose
    DevBuf A((size_t)mt * nt);
    if (left)
      permute(M, A.get(), {rows, cols}, {1, 0}, c.s);
    else
      TT_HIP(hipMemcpyAsync(A.get(), M, sizeof(double) * (size_t)mt * nt, hipMemcpyDeviceToDevice, c.s));
    if (mt > 2 * nt || (!dense_svd_left_fits_lds(mt, nt) && dense_svd_left_fits_lds(nt, nt))) {
      // T = Q R: the left vectors of T are Q times those of R (n x n)
      DevBuf Q((size_t)mt * nt), R((size_t)nt * nt), Rcm((size_t)nt * nt), Ur((size_t)nt * nt);
      qr_colmajor(A.get(), mt, nt, Q.get(), R.get(), c);
      permute(R.get(), Rcm.get(), {nt, nt}, {1, 0}, c.s);
      dense_svd_left(Rcm.get(), nt, nt, Ur.get(), sig.get(), iw, c.s);
      Gemm g;   // Ut (mt x nt col-major) = Q Ur; row-major view Ut^T = Ur^T Q^T
      g.M = nt; g.N = mt; g.K = nt;
      g.A = Ur.get(); g.am = nt; g.ak = 1;
      g.B = Q.get(); g.bk = mt; g.bn = 1;
      g.C = Ut.get(); g.cm = mt; g.cn = 1;
      gemm(g, c.s, &c.ws, GemmPrec::F64);
    } else {
      dense_svd_left(A.get(), mt, nt, Ut.get(), sig.get(), iw, c.s);
    }
  } else {
    // wide T: T^T = Q R gives T = R^T Q^T, whose left vectors are those of the
    // square R^T; the column-major R^T is the row-major R of the factorisation
    DevBuf A((size_t)nt * mt), R((size_t)mt * mt);
    if (left)
      TT_HIP(hipMemcpyAsync(A.get(), M, sizeof(double) * (size_t)nt * mt, hipMemcpyDeviceToDevice, c.s));
    else
      permute(M, A.get(), {rows, cols}, {1, 0}, c.s);
    c.dscr3.reserve((size_t)mt + 1);
    dense_qr(A.get(), nt, mt, nt, c.dscr3.get(), c.s);
    hipLaunchKernelGGL(upper_to_rowmajor_kernel, dim3(nblocks((long)mt * mt, 256)), dim3(256), 0, c.s, A.get(), nt,
                       mt, mt, R.get());
    TT_HIP(hipGetLastError());
    dense_svd_left(R.get(), mt, mt, Ut.get(), sig.get(), iw, c.s);
  }
  out.sigma.resize(k);
  TT_HIP(hipMemcpyAsync(out.sigma.data(), sig.get(), sizeof(double) * k, hipMemcpyDeviceToHost, c.s));
  if (left) {
    out.U.reserve((size_t)rows * k);       // row-major rows x k = transpose of Ut
    permute(Ut.get(), out.U.get(), {k, rows}, {1, 0}, c.s);
  } else {
    out.Vt.reserve((size_t)k * cols);      // row-major k x cols = the column-major Ut buffer
    TT_HIP(hipMemcpyAsync(out.Vt.get(), Ut.get(), sizeof(double) * (size_t)k * cols, hipMemcpyDeviceToDevice, c.s));
  }
  c.sync();
}

void orth_rows(double* G, int q, int len, Ctx& c) {
  // rows of G (q x len, row-major) = columns of a column-major len x q matrix
  if (q <= 0) return;
  DevBuf Q((size_t)len * q), R((size_t)q * q);
  qr_colmajor(G, len, q, Q.get(), R.get(), c);
  TT_HIP(hipMemcpyAsync(G, Q.get(), sizeof(double) * (size_t)len * q, hipMemcpyDeviceToDevice, c.s));
  // Q and R are recycled in stream order (no sync needed to release them)
}

void tt_orth_right(TT& t, int downto, Ctx& c) {
  const long mid = (long)t.mo * t.mi;
  for (int k = t.d - 1; k > downto; --k) {
    const int rk = t.r[k], rn = t.r[k + 1];
    const int m = (int)(mid * rn);        // rows of the column-major view (= row length of the core)
    const int n = rk;
    const int kk = std::min(m, n);
    DevBuf A((size_t)m * n), Q((size_t)m * kk), R((size_t)kk * n);
    // column-major (m x n) view of the core's row-major (rk x m) matrix is the core itself
    TT_HIP(hipMemcpyAsync(A.get(), t.core(k), sizeof(double) * (size_t)m * n, hipMemcpyDeviceToDevice, c.s));
    qr_colmajor(A.get(), m, n, Q.get(), R.get(), c);
    // new core k: Q^T as [kk][mid][rn] row-major == column-major Q buffer
    t.cores[k].reserve((size_t)kk * m);
    TT_HIP(hipMemcpyAsync(t.core(k), Q.get(), sizeof(double) * (size_t)kk * m, hipMemcpyDeviceToDevice, c.s));
    // core k-1 <- core_{k-1} R^T : [(r_{k-1} mid)][rk] x [rk][kk]
    const int rows = (int)(t.r[k - 1] * mid);
    DevBuf nc((size_t)rows * kk);
    Gemm g;
    g.M = rows; g.N = kk; g.K = rk;
    g.A = t.core(k - 1); g.am = rk; g.ak = 1;
    g.B = R.get(); g.bk = 1; g.bn = rk;          // R^T[j][c] = R[c][j]
    g.C = nc.get(); g.cm = kk; g.cn = 1;
    gemm(g, c.s, &c.ws, GemmPrec::F64);
    t.r[k] = kk;
    t.cores[k - 1].reserve((size_t)rows * kk);
    TT_HIP(hipMemcpyAsync(t.core(k - 1), nc.get(), sizeof(double) * (size_t)rows * kk, hipMemcpyDeviceToDevice, c.s));
    // the temporaries (and replaced cores) are recycled in stream order
  }
}

double tt_round_abs(TT& t, double eps, int max_rank, Ctx& c, bool* capped, double* zeta_tol) {
  if (capped) *capped = false;
  if (zeta_tol) *zeta_tol = 0.0;
  if (t.d == 1) return 0.0;
  tt_orth_right(t, 0, c);
  const double eps_k = eps / std::sqrt((double)(t.d - 1));
  const long mid = (long)t.mo * t.mi;
  double zeta2 = 0.0, zeta_tol2 = 0.0;
  for (int k = 0; k < t.d - 1; ++k) {
    const int rows = (int)(t.r[k] * mid), cols = t.r[k + 1];
    SvdOut sv;
    svd_rowmajor_side(t.core(k), rows, cols, true, sv, c);
    const int kk = sv.k;
    // smallest rank whose discarded tail is within eps_k
    std::vector<double> tail(kk + 1, 0.0);
    for (int j = kk - 1; j >= 0; --j) tail[j] = tail[j + 1] + sv.sigma[j] * sv.sigma[j];
    int rk = kk;
    for (int j = 1; j <= kk; ++j)
      if (std::sqrt(tail[j]) <= eps_k) { rk = j; break; }
    rk = std::max(1, rk);
    // the tolerance alone would discard tail[rk]; a binding cap discards more
    zeta_tol2 += tail[rk];
    if (rk > max_rank) {
      rk = max_rank;
      if (capped) *capped = true;
    }
    zeta2 += tail[rk];
    // new core k = U[:, :rk] (leading columns of the row-major U)
    DevBuf nc((size_t)rows * rk);
    copy2d(sv.U.get(), kk, nc.get(), rk, rows, rk, c.s);
    // S Vt[:rk] = U[:, :rk]^T core_k (the projection onto the kept left
    // vectors) goes into the next core: next = U[:, :rk]^T core_k core_{k+1}
    DevBuf svt((size_t)rk * cols);
    {
      Gemm g;
      g.M = rk; g.N = cols; g.K = rows;
      g.A = nc.get(); g.am = 1; g.ak = rk;
      g.B = t.core(k); g.bk = cols; g.bn = 1;
      g.C = svt.get(); g.cm = cols; g.cn = 1;
      gemm(g, c.s, &c.ws, GemmPrec::F64);
    }
    const int ncols = (int)(mid * t.r[k + 2]);
    DevBuf nn((size_t)rk * ncols);
    gemm(gemm_nn(rk, ncols, cols, svt.get(), cols, t.core(k + 1), ncols, nn.get(), ncols), c.s, &c.ws, GemmPrec::F64);
    t.r[k + 1] = rk;
    t.cores[k].reserve((size_t)rows * rk);
    TT_HIP(hipMemcpyAsync(t.core(k), nc.get(), sizeof(double) * (size_t)rows * rk, hipMemcpyDeviceToDevice, c.s));
    t.cores[k + 1].reserve((size_t)rk * ncols);
    TT_HIP(hipMemcpyAsync(t.core(k + 1), nn.get(), sizeof(double) * (size_t)rk * ncols, hipMemcpyDeviceToDevice, c.s));
    // no sync: the temporaries are recycled in stream order, and the next
    // core's SVD synchronises when it reads its singular values
  }
  if (zeta_tol) *zeta_tol = std::sqrt(zeta_tol2);
  return std::sqrt(zeta2);
}

}  // namespace ttipm
