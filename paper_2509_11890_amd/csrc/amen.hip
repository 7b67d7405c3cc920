// Block-AMEn Newton solver on the device (see amen.hpp).
//
// Per core k of a sweep:
//   1. right-hand sides: every residual term is projected onto the frame
//      with its cached environments (a projected local product whose trial is
//      the stored TT), giving R_d^, R_p^, R_c^ [, R_t^];
//   2. the reduced system of eq. (reduced_kkt_system) is solved for
//      (dX_k, dY_k [, dT_k]) — densely (LU) when small, else by restarted GMRES
//      whose matrix-free operator is the chain of projected local products;
//   3. dZ_k = Aeq^T^ dY_k [+ s Aineq^T^ dT_k] - R_d^ (local elimination);
//   4. the block core is split by SVD, the orthonormal factor becomes W_k and the
//      block index moves to the neighbour (Sec. 2.3, Block TT);
//   5. the environments of the new W_k are appended for every operator/term.
// The sweep direction alternates; the stopping test is the largest relative
// local residual of the incoming iterate over a half-sweep.
#include "amen.hpp"
#include "blocked.hpp"
#include "krylov.hpp"
#include "mlp.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <initializer_list>
#include <random>

#include "dense.hpp"
#include "ttops.hpp"

namespace ttipm {

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct EnvKey {
  const TT* op;      // nullptr: identity
  const TT* trial;   // nullptr: the frame W itself
};

struct Envs {
  std::vector<EnvKey> keys;
  std::vector<std::vector<DevBuf>> L, R;
  int d = 0;
  const TT* test = nullptr;   // nullptr: the frame W is the test TT

  int test_rank(const BlockTT& W, int bond) const { return test ? test->r[bond] : W.r[bond]; }
  const double* test_core(const BlockTT& W, int k) const { return test ? test->core(k) : W.cores[k].get(); }

  int op_rank(const EnvKey& e, int bond) const { return e.op ? e.op->r[bond] : 1; }
  int trial_rank(const EnvKey& e, const BlockTT& W, int bond) const { return e.trial ? e.trial->r[bond] : W.r[bond]; }
  const double* trial_core(const EnvKey& e, const BlockTT& W, int k) const {
    return e.trial ? e.trial->core(k) : W.cores[k].get();
  }

  void init(const std::vector<EnvKey>& ks, int d_, Ctx& c) {
    keys = ks;
    d = d_;
    L.clear();
    R.clear();
    L.resize(keys.size());
    R.resize(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
      L[i].resize(d);
      R[i].resize(d);
      L[i][0].reserve(1);
      R[i][d - 1].reserve(1);
      fill(1, 1.0, L[i][0].get(), c.s);
      fill(1, 1.0, R[i][d - 1].get(), c.s);
    }
  }

  // the steps of all keys at one core share grouped launches
  void update_left(const BlockTT& W, int k, Ctx& c) {
    std::vector<EnvStepArgs> st;
    for (size_t i = 0; i < keys.size(); ++i) {
      const EnvKey& e = keys[i];
      const int ra = test_rank(W, k), ra2 = test_rank(W, k + 1);
      const int R0 = op_rank(e, k), R1 = op_rank(e, k + 1);
      const int rc = trial_rank(e, W, k), rc2 = trial_rank(e, W, k + 1);
      L[i][k + 1].reserve((size_t)ra2 * R1 * rc2);
      st.push_back({L[i][k].get(), ra, R0, rc, test_core(W, k), 4, ra2, e.op ? e.op->core(k) : nullptr, R1, 4,
                    trial_core(e, W, k), rc2, L[i][k + 1].get()});
    }
    env_steps(st, true, c);
  }

  void update_right(const BlockTT& W, int k, Ctx& c) {
    std::vector<EnvStepArgs> st;
    for (size_t i = 0; i < keys.size(); ++i) {
      const EnvKey& e = keys[i];
      const int ra = test_rank(W, k), ra2 = test_rank(W, k + 1);
      const int R0 = op_rank(e, k), R1 = op_rank(e, k + 1);
      const int rc = trial_rank(e, W, k), rc2 = trial_rank(e, W, k + 1);
      R[i][k - 1].reserve((size_t)ra * R0 * rc);
      st.push_back({R[i][k].get(), ra2, R1, rc2, test_core(W, k), 4, ra, e.op ? e.op->core(k) : nullptr, R0, 4,
                    trial_core(e, W, k), rc, R[i][k - 1].get()});
    }
    env_steps(st, false, c);
  }
};

// The local KKT system at one core.
struct LocalKKT {
  const NewtonSys* sys;
  Envs* envs;
  const BlockTT* W;
  int k, r, s, p, L;
  int key_of_op[OP_COUNT];
  DevBuf operm[OP_COUNT];
  DevBuf tmp, tmp2;

  void setup(Ctx& c) {
    r = W->r[k];
    s = W->r[k + 1];
    p = 4 * r * s;
    L = sys->L();
    // the cores of all operators, permuted for the local products in one launch
    std::vector<PermJob> jobs;
    for (int o = 0; o < OP_COUNT; ++o) {
      if (key_of_op[o] < 0) continue;
      const TT* op = sys->ops[o];
      operm[o].reserve((size_t)op->core_size(k));
      jobs.push_back({op->core(k), operm[o].get(), {op->r[k], 4, 4, op->r[k + 1]}, {1, 3, 0, 2}});
    }
    permute_many(jobs, c.s);
    tmp.reserve(p);
    tmp2.reserve(p);
  }

  // y = alpha P_op x + beta y
  void apply(int o, const double* x, double* y, double alpha, double beta, Ctx& c) {
    const int key = key_of_op[o];
    const TT* op = sys->ops[o];
    local_apply(envs->L[key][k].get(), r, op->r[k], r, operm[o].get(), 4, envs->R[key][k].get(), s, op->r[k + 1], s,
                x, y, alpha, beta, c);
  }

  // Stage products of y = alpha P_o x + beta y for several operators, one
  // grouped launch per stage (the same three contractions as local_apply,
  // with stage buffers of each operator's own).
  struct Ap {
    int o;
    const double* x;
    double* y;
    double alpha, beta;
  };
  DevBuf gt1[OP_COUNT], gt2[OP_COUNT];

  void stages12(std::initializer_list<Ap> aps, Ctx& c) {
    Gemm s1[OP_COUNT], s2[OP_COUNT];
    int n = 0;
    for (const Ap& a : aps) {
      const TT* op = sys->ops[a.o];
      const int key = key_of_op[a.o], R = op->r[k], Rp = op->r[k + 1];
      gt1[a.o].reserve((size_t)r * R * 4 * s);
      gt2[a.o].reserve((size_t)r * 4 * Rp * s);
      // t1[(a,alpha)][(j,e)] = phiL[(a,alpha)][c] x[c][(j,e)]
      s1[n] = gemm_nn(r * R, 4 * s, r, envs->L[key][k].get(), r, a.x, 4 * s, gt1[a.o].get(), 4 * s);
      // t2[a][(i,beta)][e] = O'[(i,beta)][(alpha,j)] t1[a][(alpha,j)][e], batched over a
      Gemm& g = s2[n];
      g.M = 4 * Rp; g.N = s; g.K = R * 4; g.batch = r;
      g.A = operm[a.o].get(); g.am = (long)R * 4; g.ak = 1; g.sA = 0;
      g.B = gt1[a.o].get(); g.bk = s; g.bn = 1; g.sB = (long)R * 4 * s;
      g.C = gt2[a.o].get(); g.cm = s; g.cn = 1; g.sC = (long)4 * Rp * s;
      ++n;
    }
    gemm_grouped(s1, n, c.s, &c.ws, c.prec);
    gemm_grouped(s2, n, c.s, &c.ws, c.prec);
  }

  void stage3(std::initializer_list<Ap> aps, Ctx& c) {
    Gemm s3[OP_COUNT];
    int n = 0;
    for (const Ap& a : aps) {
      const TT* op = sys->ops[a.o];
      const int key = key_of_op[a.o], Rp = op->r[k + 1];
      // y[(a,i)][b] = alpha sum_(beta,e) t2[(a,i)][(beta,e)] phiR[b][(beta,e)] + beta y
      Gemm& g = s3[n];
      g.M = r * 4; g.N = s; g.K = Rp * s;
      g.A = gt2[a.o].get(); g.am = (long)Rp * s; g.ak = 1;
      g.B = envs->R[key][k].get(); g.bk = 1; g.bn = (long)Rp * s;
      g.C = a.y; g.cm = s; g.cn = 1;
      g.alpha = a.alpha; g.beta = a.beta;
      ++n;
    }
    gemm_grouped(s3, n, c.s, &c.ws, c.prec);
  }

  // out = K u (u, out: [L][p])
  void matvec(const double* u, double* out, Ctx& c) {
    const double* x = u;
    const double* y = u + p;
    const double sg = sys->sense;
    if (!sys->ineq) {
      // Two levels of grouped stages: every operator applied to u, then L_X
      // applied to the eliminated dZ part.  K_Y's last stage waits for the
      // second level so that no launch has two products writing one row.
      double* oc = out + (size_t)(L - 1) * p;
      stages12({{OP_AEQ, x, out, -1.0, 0.0}, {OP_KY, y, out, 1.0, 1.0}, {OP_AEQT, y, tmp.get(), 1.0, 0.0},
                {OP_LZ, x, oc, 1.0, 0.0}}, c);
      stage3({{OP_AEQ, x, out, -1.0, 0.0}, {OP_AEQT, y, tmp.get(), 1.0, 0.0}, {OP_LZ, x, oc, 1.0, 0.0}}, c);
      stages12({{OP_LX, tmp.get(), oc, 1.0, 1.0}}, c);
      stage3({{OP_LX, tmp.get(), oc, 1.0, 1.0}, {OP_KY, y, out, 1.0, 1.0}}, c);
      return;
    }
    // row p
    apply(OP_AEQ, x, out, -1.0, 0.0, c);
    apply(OP_KY, y, out, 1.0, 1.0, c);
    double* oc = out + (size_t)(L - 1) * p;
    // chained dZ part: tmp = Aeq^T^ y (+ s Aineq^T^ t)
    apply(OP_AEQT, y, tmp.get(), 1.0, 0.0, c);
    if (sys->ineq) {
      const double* t = u + 2 * p;
      double* ot = out + p;
      apply(OP_TA, x, ot, -sg, 0.0, c);
      apply(OP_DK, t, ot, 1.0, 1.0, c);
      apply(OP_AIT, t, tmp.get(), sg, 1.0, c);
    }
    apply(OP_LZ, x, oc, 1.0, 0.0, c);
    apply(OP_LX, tmp.get(), oc, 1.0, 1.0, c);
  }
};

__global__ void scale_components_kernel(const double* in, double* out, int Lp, int r, int m, int s,
                                        const double* w) {
  // in [l][a][i][b] -> out [a][i][l][b] scaled by 1/w[l]
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)Lp * r * m * s;
  if (t >= total) return;
  long q = t;
  int b = (int)(q % s); q /= s;
  int i = (int)(q % m); q /= m;
  int a = (int)(q % r); q /= r;
  int l = (int)q;
  out[(((long)a * m + i) * Lp + l) * s + b] = in[t] / w[l];
}

__global__ void scale_components_right_kernel(const double* in, double* out, int Lp, int r, int m, int s,
                                              const double* w) {
  // in [l][a][i][b] -> out [a][l][i][b] scaled by 1/w[l]
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long total = (long)Lp * r * m * s;
  if (t >= total) return;
  long q = t;
  int b = (int)(q % s); q /= s;
  int i = (int)(q % m); q /= m;
  int a = (int)(q % r); q /= r;
  int l = (int)q;
  out[(((long)a * Lp + l) * m + i) * s + b] = in[t] / w[l];
}

int rank_for(const std::vector<double>& sv, double tol_rel, int cap) {
  double tot = 0.0;
  for (double x : sv) tot += x * x;
  if (tot == 0.0) return 1;
  const int n = (int)sv.size();
  std::vector<double> tail(n + 1, 0.0);
  for (int j = n - 1; j >= 0; --j) tail[j] = tail[j + 1] + sv[j] * sv[j];
  int rk = n;
  for (int j = 1; j < n; ++j)
    if (std::sqrt(tail[j]) <= tol_rel * std::sqrt(tot)) { rk = j; break; }
  return std::max(1, std::min(rk, cap));
}

// host copy of device vector norms per component
std::vector<double> component_norms(const double* blk, int Lp, long n, Ctx& c) {
  c.dot_out.reserve(Lp);
  c.dot_part.reserve(mdot_part_size(1));
  std::vector<double> out(Lp);
  double* h = c.host(Lp);
  for (int l = 0; l < Lp; ++l) mdot(n, 1, blk + (long)l * n, n, blk + (long)l * n, c.dot_out.get() + l, c.dot_part.get(), c.s);
  TT_HIP(hipMemcpyAsync(h, c.dot_out.get(), sizeof(double) * Lp, hipMemcpyDeviceToHost, c.s));
  c.sync();
  for (int l = 0; l < Lp; ++l) out[l] = std::sqrt(std::max(h[l], 0.0));
  return out;
}

}  // namespace

double dev_norm(const double* x, long n, Ctx& c) {
  c.dot_out.reserve(1);
  c.dot_part.reserve(mdot_part_size(1));
  mdot(n, 1, x, n, x, c.dot_out.get(), c.dot_part.get(), c.s);
  double* h = c.host(1);
  TT_HIP(hipMemcpyAsync(h, c.dot_out.get(), sizeof(double), hipMemcpyDeviceToHost, c.s));
  c.sync();
  return std::sqrt(std::max(h[0], 0.0));
}

// n x q block of seeded standard normal numbers (row-major), uploaded to dev.
static void random_block(double* dev, long count, unsigned long long seed, Ctx& c) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> h(count);
  for (double& x : h) x = nd(rng);
  TT_HIP(hipMemcpyAsync(dev, h.data(), sizeof(double) * count, hipMemcpyHostToDevice, c.s));
  c.sync();
}

void random_orth_rows(const double* B, int q0, long bj, long bi, int len, double* G, int q, unsigned long long seed,
                      Ctx& c) {
  if (q <= 0) return;
  random_block(G, (long)q * len, seed, c);
  if (q0 > 0) {
    DevBuf T((size_t)q * q0);
    for (int pass = 0; pass < 2; ++pass) {
      Gemm g1;   // T = G B^T  (q x q0)
      g1.M = q; g1.N = q0; g1.K = len;
      g1.A = G; g1.am = len; g1.ak = 1;
      g1.B = B; g1.bk = bi; g1.bn = bj;
      g1.C = T.get(); g1.cm = q0; g1.cn = 1;
      gemm(g1, c.s, &c.ws, GemmPrec::F64);
      Gemm g2;   // G -= T B
      g2.M = q; g2.N = len; g2.K = q0;
      g2.A = T.get(); g2.am = q0; g2.ak = 1;
      g2.B = B; g2.bk = bj; g2.bn = bi;
      g2.C = G; g2.cm = len; g2.cn = 1;
      g2.alpha = -1.0; g2.beta = 1.0;
      gemm(g2, c.s, &c.ws, GemmPrec::F64);
    }
  }
  orth_rows(G, q, len, c);
}

// G (q x len) = the q leading principal directions of the ncand candidate
// rows C (q x len row-major, ncand x len) after their components along the q0
// orthonormal vectors b_j (B[j*bj + i*bi]) are removed (two passes): the right
// singular vectors of the projected candidates with the largest singular
// values, orthonormal and orthogonal to the b_j.  Directions the candidates do
// not supply (rank below q) are filled with seeded random ones.
void principal_orth_rows(const double* B, int q0, long bj, long bi, int len, const double* C, int ncand, double* G,
                         int q, unsigned long long seed, Ctx& c) {
  if (q <= 0) return;
  DevBuf P((size_t)ncand * len);
  TT_HIP(hipMemcpyAsync(P.get(), C, sizeof(double) * (size_t)ncand * len, hipMemcpyDeviceToDevice, c.s));
  auto project = [&](double* M, int nr) {
    if (q0 <= 0) return;
    DevBuf T((size_t)nr * q0);
    for (int pass = 0; pass < 2; ++pass) {
      Gemm g1;   // T = M B^T
      g1.M = nr; g1.N = q0; g1.K = len;
      g1.A = M; g1.am = len; g1.ak = 1;
      g1.B = B; g1.bk = bi; g1.bn = bj;
      g1.C = T.get(); g1.cm = q0; g1.cn = 1;
      gemm(g1, c.s, &c.ws, GemmPrec::F64);
      Gemm g2;   // M -= T B
      g2.M = nr; g2.N = len; g2.K = q0;
      g2.A = T.get(); g2.am = q0; g2.ak = 1;
      g2.B = B; g2.bk = bj; g2.bn = bi;
      g2.C = M; g2.cm = len; g2.cn = 1;
      g2.alpha = -1.0; g2.beta = 1.0;
      gemm(g2, c.s, &c.ws, GemmPrec::F64);
    }
  };
  project(P.get(), ncand);
  SvdOut sv;
  svd_rowmajor_side(P.get(), ncand, len, false, sv, c);
  // directions with a singular value above rounding level are taken
  int take = 0;
  const double s0 = sv.sigma.empty() ? 0.0 : sv.sigma[0];
  while (take < std::min(q, sv.k) && sv.sigma[take] > 1e-12 * s0 && s0 > 0.0) ++take;
  if (take > 0)
    TT_HIP(hipMemcpyAsync(G, sv.Vt.get(), sizeof(double) * (size_t)take * len, hipMemcpyDeviceToDevice, c.s));
  if (take < q) {
    // random rows orthogonal to the b_j and to the directions taken
    DevBuf Bx((size_t)(q0 + take) * len);
    if (q0 > 0) {
      if (bi == 1) {
        copy2d(B, bj, Bx.get(), len, q0, len, c.s);
      } else {
        TT_REQUIRE(bj == 1, "basis vectors must be rows or columns");
        DevBuf t((size_t)len * q0);
        copy2d(B, bi, t.get(), q0, len, q0, c.s);
        permute(t.get(), Bx.get(), {len, q0}, {1, 0}, c.s);
      }
    }
    if (take > 0)
      TT_HIP(hipMemcpyAsync(Bx.get() + (size_t)q0 * len, G, sizeof(double) * (size_t)take * len,
                            hipMemcpyDeviceToDevice, c.s));
    random_orth_rows(Bx.get(), q0 + take, len, 1, len, G + (size_t)take * len, q - take, seed, c);
  }
}

// Move the block index from W.pos to W.pos + 1 (dir > 0) or W.pos - 1 (dir < 0).

bool split_block(BlockTT& W, int dir, double tol_rel, int cap, Ctx& c, int kick, unsigned long long seed,
                 const CandidateFn* cand_fn) {
  bool capped = false;
  const int k = W.pos, Lp = W.Lp, r = W.r[k], s = W.r[k + 1], md = W.m;
  const long n1 = (long)r * md * s;
  // Components are normalised before the SVD so that a small component is not
  // truncated away next to a large one; a component at rounding level (e.g. a
  // Newton block whose right-hand side vanishes) keeps the largest weight, so
  // that its noise is not amplified into spurious rank.
  std::vector<double> w = component_norms(W.blk.get(), Lp, n1, c);
  double wmax = 0.0;
  for (double x : w) wmax = std::max(wmax, x);
  for (double& x : w) x = (wmax == 0.0) ? 1.0 : (x > 1e-8 * wmax ? x : wmax);
  DevBuf wdev(Lp);
  TT_HIP(hipMemcpyAsync(wdev.get(), w.data(), sizeof(double) * Lp, hipMemcpyHostToDevice, c.s));
  const long total = (long)Lp * n1;
  DevBuf Ms(total), M(total);
  DevBuf ones(Lp);
  fill(Lp, 1.0, ones.get(), c.s);
  if (dir > 0) {
    // M[(a,i)][(l,b)]
    const int rows = md * r, cols = Lp * s;
    hipLaunchKernelGGL(scale_components_kernel, dim3(nblocks(total, 256)), dim3(256), 0, c.s, W.blk.get(), Ms.get(),
                       Lp, r, md, s, wdev.get());
    hipLaunchKernelGGL(scale_components_kernel, dim3(nblocks(total, 256)), dim3(256), 0, c.s, W.blk.get(), M.get(),
                       Lp, r, md, s, ones.get());
    TT_HIP(hipGetLastError());
    SvdOut sv;
    svd_rowmajor_side(Ms.get(), rows, cols, true, sv, c);
    // Enrichment fills only the capacity the rank cap leaves: once the cap
    // binds, the truncated SVD directions are kept in full.
    const int rk_tol = rank_for(sv.sigma, tol_rel, sv.k);
    const int rk0 = std::max(1, std::min(rk_tol, cap));
    capped = rk_tol > cap;
    const int q = std::max(0, std::min({kick, rows - rk0, cap - rk0}));
    const int rk = rk0 + q;
    const double* cand = nullptr;
    int ncand = 0;
    if (q > 0 && cand_fn) ncand = (*cand_fn)(&cand);
    // W_k = [U[:, :rk0] | kick]  ([r][4][rk])
    W.cores[k].reserve((size_t)rows * rk);
    copy2d(sv.U.get(), sv.k, W.cores[k].get(), rk, rows, rk0, c.s);
    if (q > 0) {
      // enrichment columns orthonormalised against U (the columns of W_k)
      DevBuf G((size_t)q * rows);                                // G^T: q x rows
      if (ncand > 0)
        principal_orth_rows(W.cores[k].get(), rk0, 1, rk, rows, cand, ncand, G.get(), q, seed, c);
      else
        random_orth_rows(W.cores[k].get(), rk0, 1, rk, rows, G.get(), q, seed, c);
      // columns rk0.. of W_k = G (transposed)
      DevBuf Gt((size_t)rows * q);
      permute(G.get(), Gt.get(), {q, rows}, {1, 0}, c.s);
      copy2d(Gt.get(), q, W.cores[k].get() + rk0, rk, rows, q, c.s);
    }
    // coef = U_k^T M  (rk x (l,b))
    DevBuf coef((size_t)rk * cols);
    Gemm g;
    g.M = rk; g.N = cols; g.K = rows;
    g.A = W.cores[k].get(); g.am = 1; g.ak = rk;
    g.B = M.get(); g.bk = cols; g.bn = 1;
    g.C = coef.get(); g.cm = cols; g.cn = 1;
    gemm(g, c.s, &c.ws, GemmPrec::F64);
    // new block at k+1: [(c,l)][(i,t)] = coef[(c,l)][b] W_{k+1}[b][(i,t)] -> permute to [l][c][i][t]
    const int t = W.r[k + 2];
    DevBuf nb((size_t)rk * Lp * md * t);
    gemm(gemm_nn(rk * Lp, md * t, s, coef.get(), s, W.cores[k + 1].get(), md * t, nb.get(), md * t), c.s, &c.ws,
         GemmPrec::F64);
    W.blk.reserve((size_t)Lp * rk * md * t);
    permute(nb.get(), W.blk.get(), {rk, Lp, md, t}, {1, 0, 2, 3}, c.s);
    W.r[k + 1] = rk;
    W.pos = k + 1;
  } else {
    // M[(a,l)][(i,b)]
    const int rows = r * Lp, cols = md * s;
    hipLaunchKernelGGL(scale_components_right_kernel, dim3(nblocks(total, 256)), dim3(256), 0, c.s, W.blk.get(),
                       Ms.get(), Lp, r, md, s, wdev.get());
    hipLaunchKernelGGL(scale_components_right_kernel, dim3(nblocks(total, 256)), dim3(256), 0, c.s, W.blk.get(),
                       M.get(), Lp, r, md, s, ones.get());
    TT_HIP(hipGetLastError());
    SvdOut sv;
    svd_rowmajor_side(Ms.get(), rows, cols, false, sv, c);
    const int rk_tol = rank_for(sv.sigma, tol_rel, sv.k);
    const int rk0 = std::max(1, std::min(rk_tol, cap));
    capped = rk_tol > cap;
    const int q = std::max(0, std::min({kick, cols - rk0, cap - rk0}));
    const int rk = rk0 + q;
    const double* cand = nullptr;
    int ncand = 0;
    if (q > 0 && cand_fn) ncand = (*cand_fn)(&cand);
    // W_k = [Vt[:rk0]; kick]  ([rk][4][s])
    W.cores[k].reserve((size_t)rk * cols);
    TT_HIP(hipMemcpyAsync(W.cores[k].get(), sv.Vt.get(), sizeof(double) * (size_t)rk0 * cols, hipMemcpyDeviceToDevice,
                          c.s));
    if (q > 0) {   // enrichment rows orthonormalised against those of Vt
      if (ncand > 0)
        principal_orth_rows(W.cores[k].get(), rk0, cols, 1, cols, cand, ncand, W.cores[k].get() + (size_t)rk0 * cols,
                            q, seed, c);
      else
        random_orth_rows(W.cores[k].get(), rk0, cols, 1, cols, W.cores[k].get() + (size_t)rk0 * cols, q, seed, c);
    }
    // coef = M Vt[:rk]^T  ((a,l) x rk)
    DevBuf coef((size_t)rows * rk);
    Gemm g;
    g.M = rows; g.N = rk; g.K = cols;
    g.A = M.get(); g.am = cols; g.ak = 1;
    g.B = W.cores[k].get(); g.bk = 1; g.bn = cols;
    g.C = coef.get(); g.cm = rk; g.cn = 1;
    gemm(g, c.s, &c.ws, GemmPrec::F64);
    // new block at k-1: [(q,i)][(l,c)] = W_{k-1}[(q,i)][a] coef[a][(l,c)] -> permute to [l][q][i][c]
    const int rq = W.r[k - 1];
    DevBuf nb((size_t)rq * md * Lp * rk);
    gemm(gemm_nn(rq * md, Lp * rk, r, W.cores[k - 1].get(), r, coef.get(), Lp * rk, nb.get(), Lp * rk), c.s, &c.ws,
         GemmPrec::F64);
    W.blk.reserve((size_t)Lp * rq * md * rk);
    permute(nb.get(), W.blk.get(), {rq, md, Lp, rk}, {2, 0, 1, 3}, c.s);
    W.r[k] = rk;
    W.pos = k - 1;
  }
  // no sync: the temporaries are recycled in stream order, and everything the
  // host decides on (ranks, the cap) is already on the host
  return capped;
}

namespace {

// frames above this size use the blocked dense factorisations
constexpr int kBlockedMin = 192;

// ---------------------------------------------------------------------------
// local solvers
// ---------------------------------------------------------------------------

// Dense direct solve of the reduced system.
void solve_direct(LocalKKT& K, const double* f, double* u, Ctx& c) {
  const int p = K.p, L = K.L;
  const NewtonSys& sys = *K.sys;
  auto dense = [&](int o, DevBuf& out) {
    const TT* op = sys.ops[o];
    const int key = K.key_of_op[o];
    out.reserve((size_t)p * p);
    local_dense_op(K.envs->L[key][K.k].get(), K.r, op->r[K.k], op->core(K.k), 4, K.envs->R[key][K.k].get(), K.s,
                   op->r[K.k + 1], out.get(), c);
  };
  DevBuf A, AT, KY, LZ, LX, LXAT;
  dense(OP_AEQ, A);
  dense(OP_AEQT, AT);
  dense(OP_KY, KY);
  dense(OP_LZ, LZ);
  dense(OP_LX, LX);
  LXAT.reserve((size_t)p * p);
  gemm(gemm_nn(p, p, p, LX.get(), p, AT.get(), p, LXAT.get(), p), c.s, &c.ws, GemmPrec::F64);
  const int N = L * p;
  DevBuf Kd((size_t)N * N), rhs(N);
  fill((long)N * N, 0.0, Kd.get(), c.s);
  auto put = [&](const double* blk, int bi, int bj, double alpha) {
    place_block(blk, p, 1, p, Kd.get() + (size_t)bi * p * N, p, N, 0, bj * p, alpha, c.s);
  };
  // place_block writes [n0][mid][n1] into [N0][mid][N1]; rows are strided by N here
  put(A.get(), 0, 0, -1.0);
  put(KY.get(), 0, 1, 1.0);
  put(LZ.get(), L - 1, 0, 1.0);
  put(LXAT.get(), L - 1, 1, 1.0);
  if (sys.ineq) {
    DevBuf TA, DK, AiT, LXAiT;
    dense(OP_TA, TA);
    dense(OP_DK, DK);
    dense(OP_AIT, AiT);
    LXAiT.reserve((size_t)p * p);
    gemm(gemm_nn(p, p, p, LX.get(), p, AiT.get(), p, LXAiT.get(), p), c.s, &c.ws, GemmPrec::F64);
    put(TA.get(), 1, 0, -sys.sense);
    put(DK.get(), 1, 2, 1.0);
    put(LXAiT.get(), 2, 2, sys.sense);
    c.sync();
  }
  TT_HIP(hipMemcpyAsync(rhs.get(), f, sizeof(double) * N, hipMemcpyDeviceToDevice, c.s));
  c.ired.reserve(4);
  int* st = reinterpret_cast<int*>(c.ired.get());
  int hst = 0;
  if (N > kBlockedMin) {
    BlockedFactors fk;
    hst = lu_blocked(Kd.get(), N, fk, c);
    if (hst == 0) lu_solve_blocked(Kd.get(), N, fk, rhs.get(), 1, c);
  } else {
    dense_lu_solve(Kd.get(), N, rhs.get(), 1, st, c.s);
    TT_HIP(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, c.s));
  }
  c.sync();
  if (hst != 0) throw Error(TT_ERR_NUMERIC, "singular local KKT system (zero pivot)");
  TT_HIP(hipMemcpyAsync(u, rhs.get(), sizeof(double) * N, hipMemcpyDeviceToDevice, c.s));
}

// Direct solve by the block elimination of Sec. 3.3 (systems without
// inequalities): Cholesky of L_Z^, the Schur complement
//   S = Aeq^ L_Z^{-1} L_X^ Aeq^T^ + K_Y^,   S dY = Aeq^ L_Z^{-1}(L_X^ R_d^ - R_c^) - R_p^,
// then dZ = Aeq^T^ dY - R_d^ and dX = -L_Z^{-1}(R_c^ + L_X^ dZ).  Unlike an LU of
// the whole unsymmetric block system, the ill-conditioning of L_Z^ and L_X^
// as mu -> 0 stays inside the Cholesky solves.  Returns false if L_Z^ is not
// numerically positive definite (the caller then falls back to the LU).
bool solve_elim(LocalKKT& K, const double* Rd, const double* Rp, const double* Rc, double* u, Ctx& c) {
  const int p = K.p;
  const NewtonSys& sys = *K.sys;
  auto dense = [&](int o, DevBuf& out) {
    const TT* op = sys.ops[o];
    const int key = K.key_of_op[o];
    out.reserve((size_t)p * p);
    local_dense_op(K.envs->L[key][K.k].get(), K.r, op->r[K.k], op->core(K.k), 4, K.envs->R[key][K.k].get(), K.s,
                   op->r[K.k + 1], out.get(), c);
  };
  DevBuf A, AT, KY, LZ, LX, T1, S, v1, v2, ry;
  dense(OP_LZ, LZ);
  dense_symmetrize(LZ.get(), p, c.s);
  c.ired.reserve(4);
  int* st = reinterpret_cast<int*>(c.ired.get());
  // Frames whose matrices fit one workgroup's LDS go through the LDS-resident
  // single-workgroup kernels (fewest launches); larger ones through the
  // blocked (GEMM-based) factorisations.
  const bool blocked = p > kBlockedMin || !dense_small_fits_lds(p);
  BlockedFactors fz, fs;
  int hst = 0;
  if (blocked) {
    hst = chol_blocked(LZ.get(), p, fz, c);
    if (hst != 0) return false;
  } else {
    // The status (st[0]) is read back with the LU's (st[1]) at the end, so the
    // stream does not stop here: a failed factorisation only wastes the work
    // queued after it, and the caller then solves the whole block system.
    dense_cholesky(LZ.get(), p, st, c.s);
  }
  dense(OP_AEQ, A);
  dense(OP_AEQT, AT);
  dense(OP_KY, KY);
  dense(OP_LX, LX);
  auto solve_LZ = [&](double* B, int nrhs) {   // B <- L_Z^{-1} B = L^{-T} L^{-1} B
    if (blocked) {
      trsm_blocked(LZ.get(), p, fz, B, nrhs, false, c);
      trsm_blocked(LZ.get(), p, fz, B, nrhs, true, c);
    } else {
      dense_chol_solve(LZ.get(), p, B, nrhs, c.s);
    }
  };
  // G = L_Z^{-1} L_X^ Aeq^T^ ; S = Aeq^ G + K_Y^ ;
  // rhs_y = Aeq^ L_Z^{-1}(L_X^ R_d^ - R_c^) - R_p^.
  // With the single-workgroup solves, the p columns of L_X^ Aeq^T^ and the
  // vector L_X^ R_d^ - R_c^ go through one triangular-solve launch as the
  // independent columns of one p x (p + 1) buffer (the solve's latency does
  // not depend on the number of columns; each column's arithmetic is the same).
  const int tw = blocked ? p : p + 1;
  T1.reserve((size_t)p * tw);
  v1.reserve(p);
  v2.reserve(p);
  gemm(gemm_nn(p, p, p, LX.get(), p, AT.get(), p, T1.get(), tw), c.s, &c.ws, GemmPrec::F64);
  if (blocked) solve_LZ(T1.get(), p);
  gemm(gemm_nn(p, 1, p, LX.get(), p, Rd, 1, v1.get(), 1), c.s, &c.ws, GemmPrec::F64);
  axpby(p, -1.0, Rc, 1.0, v1.get(), c.s);
  if (blocked) {
    solve_LZ(v1.get(), 1);
  } else {
    copy2d(v1.get(), 1, T1.get() + p, tw, p, 1, c.s);
    solve_LZ(T1.get(), p + 1);
    copy2d(T1.get() + p, tw, v1.get(), 1, p, 1, c.s);
  }
  S.reserve((size_t)p * p);
  TT_HIP(hipMemcpyAsync(S.get(), KY.get(), sizeof(double) * (size_t)p * p, hipMemcpyDeviceToDevice, c.s));
  gemm(gemm_nn(p, p, p, A.get(), p, T1.get(), tw, S.get(), p, 1.0, 1.0), c.s, &c.ws, GemmPrec::F64);
  ry.reserve(p);
  gemm(gemm_nn(p, 1, p, A.get(), p, v1.get(), 1, ry.get(), 1), c.s, &c.ws, GemmPrec::F64);
  axpby(p, -1.0, Rp, 1.0, ry.get(), c.s);
  if (blocked) {
    hst = lu_blocked(S.get(), p, fs, c);
    if (hst == 0) lu_solve_blocked(S.get(), p, fs, ry.get(), 1, c);
  } else {
    dense_lu_solve(S.get(), p, ry.get(), 1, st + 1, c.s);
  }
  if (hst != 0) throw Error(TT_ERR_NUMERIC, "singular Schur complement in the local block elimination");
  // dZ = Aeq^T^ y - R_d^ ; dX = -L_Z^{-1}(R_c^ + L_X^ dZ)
  gemm(gemm_nn(p, 1, p, AT.get(), p, ry.get(), 1, v1.get(), 1), c.s, &c.ws, GemmPrec::F64);
  axpby(p, -1.0, Rd, 1.0, v1.get(), c.s);
  TT_HIP(hipMemcpyAsync(v2.get(), Rc, sizeof(double) * p, hipMemcpyDeviceToDevice, c.s));
  gemm(gemm_nn(p, 1, p, LX.get(), p, v1.get(), 1, v2.get(), 1, 1.0, 1.0), c.s, &c.ws, GemmPrec::F64);
  solve_LZ(v2.get(), 1);
  axpby(p, -1.0, v2.get(), 0.0, u, c.s);
  TT_HIP(hipMemcpyAsync(u + p, ry.get(), sizeof(double) * p, hipMemcpyDeviceToDevice, c.s));
  if (!blocked) {
    int hs[2] = {0, 0};
    TT_HIP(hipMemcpyAsync(hs, st, sizeof(hs), hipMemcpyDeviceToHost, c.s));
    c.sync();
    if (hs[0] != 0) return false;
    if (hs[1] != 0) throw Error(TT_ERR_NUMERIC, "singular Schur complement in the local block elimination");
  }
  c.sync();
  return true;
}

// Raw (not inverted) block-Jacobi blocks of the reduced local system.
void build_block_jacobi(LocalKKT& K, BlockJacobi& bj, Ctx& c) {
  const NewtonSys& sys = *K.sys;
  auto op = [&](int o) {
    const TT* t = sys.ops[o];
    const int key = K.key_of_op[o];
    return BlockJacobi::Op{K.envs->L[key][K.k].get(), t->core(K.k), K.envs->R[key][K.k].get(), t->r[K.k],
                           t->r[K.k + 1]};
  };
  const int L = K.L;
  const double sg = sys.sense;
  bj.init(K.r, K.s, 4, L, c);
  BlockJacobi::Op o1 = op(OP_AEQ);
  bj.add(0, 0, -1.0, &o1, 1, c);
  o1 = op(OP_KY);
  bj.add(0, 1, 1.0, &o1, 1, c);
  o1 = op(OP_LZ);
  bj.add(L - 1, 0, 1.0, &o1, 1, c);
  BlockJacobi::Op ch[2] = {op(OP_AEQT), op(OP_LX)};
  bj.add(L - 1, 1, 1.0, ch, 2, c);
  if (sys.ineq) {
    o1 = op(OP_TA);
    bj.add(1, 0, -sg, &o1, 1, c);
    o1 = op(OP_DK);
    bj.add(1, 2, 1.0, &o1, 1, c);
    BlockJacobi::Op ch2[2] = {op(OP_AIT), op(OP_LX)};
    bj.add(L - 1, 2, sg, ch2, 2, c);
  }
}

void mlp_context(const LocalKKT& K, const AmenParams& prm, float ctx[4]) {
  ctx[0] = (float)std::log10(std::max(prm.mu, 1e-300));
  ctx[1] = (float)K.k / (float)std::max(1, K.W->d);
  ctx[2] = (float)K.r / 64.f;
  ctx[3] = (float)K.s / 64.f;
}

// Matrix-free local solve by restarted GMRES (krylov.hip): optionally right
// preconditioned by the block-Jacobi inverse of the (a, b) diagonal blocks of
// the reduced system, or by the learned correction of it (MLP), and in mixed
// mode with BF16-operand Arnoldi products and FP64 residual refinement at
// every restart.  Fallback rule of the MLP preconditioner: at each core the
// first solve of an AMEn call uses block Jacobi and records its iteration
// count; later solves try the MLP with that count as the iteration budget and
// redo the solve with block Jacobi when it is not met.
int solve_gmres(LocalKKT& K, const double* f, double* u, const AmenParams& prm, std::vector<int>& bj_ref,
                AmenInfo& info, double* rel_res, Ctx& c) {
  const long n = (long)K.L * K.p;
  KrylovOps ops;
  ops.matvec = [&](const double* x, double* y, bool low) {
    c.prec = low ? GemmPrec::BF16 : GemmPrec::F64;
    K.matvec(x, y, c);
    c.prec = GemmPrec::F64;
  };
  KrylovParams kp;
  // the local solve is taken a factor 4 below the sweep's residual target
  // (tol = eta/2): tighter solves only cost Krylov steps (a factor 10 took
  // 8 % longer on the rank-32 MaxCut frames with the same iterates)
  kp.rtol = std::max(prm.tol * 0.25, 1e-14);
  kp.restart = prm.gmres_restart;
  kp.maxit = prm.gmres_maxit;
  kp.mixed = prm.mixed;
  KrylovInfo ki;
  if (prm.precond == TT_PREC_NONE) {
    gmres_solve(n, ops, f, u, kp, ki, c);
    *rel_res = ki.rel_res;
    return ki.iters;
  }
  BlockJacobi raw, bj;
  build_block_jacobi(K, raw, c);
  bj.copy_from(raw, c);
  bj.invert(c);
  ops.precond = [&](const double* x, double* y) { bj.apply(x, y, c); };
  const bool try_mlp = prm.precond == TT_PREC_MLP && prm.mlp && bj_ref[K.k] > 0;
  if (try_mlp) {
    DevBuf u0(n);
    TT_HIP(hipMemcpyAsync(u0.get(), u, sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
    BlockJacobi ml;
    ml.copy_from(bj, c);
    float ctx[4];
    mlp_context(K, prm, ctx);
    mlp_correct_blocks(*prm.mlp, raw, ml, ctx, c);
    KrylovOps mops = ops;
    mops.precond = [&](const double* x, double* y) { ml.apply(x, y, c); };
    KrylovParams mp = kp;
    mp.maxit = std::min(kp.maxit, bj_ref[K.k]);
    gmres_solve(n, mops, f, u, mp, ki, c);
    if (ki.rel_res <= kp.rtol) {
      info.mlp_used++;
      *rel_res = ki.rel_res;
      return ki.iters;
    }
    info.mlp_fallbacks++;
    TT_HIP(hipMemcpyAsync(u, u0.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
    const int spent = ki.iters;
    gmres_solve(n, ops, f, u, kp, ki, c);
    bj_ref[K.k] = std::max(1, ki.iters);
    *rel_res = ki.rel_res;
    return ki.iters + spent;
  }
  gmres_solve(n, ops, f, u, kp, ki, c);
  bj_ref[K.k] = std::max(1, ki.iters);
  *rel_res = ki.rel_res;
  return ki.iters;
}

__global__ void stack_dz_kernel(double* dz, const double* tmp, const double* rd, long p) {
  long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < p) dz[t] = tmp[t] - rd[t];
}

}  // namespace

// ---------------------------------------------------------------------------
// dense projected operator (for the direct solve and the public ABI)
// ---------------------------------------------------------------------------
void local_dense_ops(const std::vector<DenseOpArgs>& v, Ctx& c) {
  std::vector<DevBuf> T1(v.size()), T2(v.size());
  std::vector<Gemm> g1, g2;
  for (size_t q = 0; q < v.size(); ++q) {
    const DenseOpArgs& a = v[q];
    // T1[a][c][(i,j,beta)] = sum_alpha phiL[a][alpha][c] O[alpha][(i,j,beta)]
    const long w = (long)a.m * a.m * a.Rp;
    T1[q].reserve((size_t)a.r * a.r * w);
    T2[q].reserve((size_t)a.r * a.r * a.m * a.m * a.s * a.s);
    Gemm g;
    g.M = a.r; g.N = (int)w; g.K = a.R; g.batch = a.r;
    g.A = a.phiL; g.am = 1; g.ak = a.r; g.sA = (long)a.R * a.r;
    g.B = a.O; g.bk = w; g.bn = 1; g.sB = 0;
    g.C = T1[q].get(); g.cm = w; g.cn = 1; g.sC = (long)a.r * w;
    g1.push_back(g);
    // T2[(a,c,i,j)][b][e] = sum_beta T1[(a,c,i,j)][beta] phiR[b][beta][e]
    Gemm h;
    h.M = a.r * a.r * a.m * a.m; h.N = a.s; h.K = a.Rp; h.batch = a.s;
    h.A = T1[q].get(); h.am = a.Rp; h.ak = 1; h.sA = 0;
    h.B = a.phiR; h.bk = a.s; h.bn = 1; h.sB = (long)a.Rp * a.s;
    h.C = T2[q].get(); h.cm = (long)a.s * a.s; h.cn = 1; h.sC = a.s;
    g2.push_back(h);
  }
  gemm_grouped(g1.data(), (int)g1.size(), c.s, &c.ws, GemmPrec::F64);
  gemm_grouped(g2.data(), (int)g2.size(), c.s, &c.ws, GemmPrec::F64);
  // [a][c][i][j][b][e] -> [a][i][b][c][j][e]
  for (size_t q = 0; q < v.size(); ++q) {
    const DenseOpArgs& a = v[q];
    permute(T2[q].get(), a.out, {a.r, a.r, a.m, a.m, a.s, a.s}, {0, 2, 4, 1, 3, 5}, c.s);
  }
  // no sync: the stage buffers go back to this stream's free list, whose
  // blocks later work on the same stream reuses only after these kernels
}

void local_dense_op(const double* phiL, int r, int R, const double* O, int m, const double* phiR, int s, int Rp,
                    double* out, Ctx& c) {
  local_dense_ops({{phiL, r, R, O, m, phiR, s, Rp, out}}, c);
}

TT BlockTT::component(int l, Ctx& c) const {
  TT t(d, m, 1);
  t.r = r;
  for (int k = 0; k < d; ++k) {
    t.alloc(k);
    const double* src = (k == pos) ? blk.get() + (size_t)l * r[k] * m * r[k + 1] : cores[k].get();
    TT_HIP(hipMemcpyAsync(t.core(k), src, sizeof(double) * t.core_size(k), hipMemcpyDeviceToDevice, c.s));
  }
  return t;
}

BlockTT block_from_frame(const TT& frame, int Lp, Ctx& c) {
  TT f = tt_clone(frame, c);
  tt_orth_right(f, 0, c);
  BlockTT W;
  W.d = f.d;
  W.Lp = Lp;
  W.m = f.mo * f.mi;
  W.pos = 0;
  W.r = f.r;
  W.cores.resize(f.d);
  for (int k = 1; k < f.d; ++k) W.cores[k] = std::move(f.cores[k]);
  W.blk.reserve((size_t)Lp * W.m * W.r[1]);
  fill((long)Lp * W.m * W.r[1], 0.0, W.blk.get(), c.s);
  return W;
}

void newton_residual(const NewtonSys& sys, const BlockTT& W, double* res, double* rhs, Ctx& c, ResidualRhs* rr) {
  struct Img {
    double coef;
    const TT* op;   // nullptr: identity
    const TT* vec;
  };
  const int L = sys.L();
  std::vector<TT> comp;
  for (int l = 0; l <= L; ++l) comp.push_back(W.component(l, c));
  const TT& dX = comp[0];
  const TT& dY = comp[1];
  const TT& dZ = comp[L];
  const TT* dT = sys.ineq ? &comp[2] : nullptr;
  std::vector<Img> R[4], KU[4];
  for (const Term& t : sys.terms) R[t.res].push_back({t.coef, t.op >= 0 ? sys.ops[t.op] : nullptr, t.vec});
  // K dU, block rows of eq. (tt-kkt-newton-system)
  KU[RES_D] = {{1.0, nullptr, &dZ}, {-1.0, sys.ops[OP_AEQT], &dY}};
  if (sys.ineq) KU[RES_D].push_back({-sys.sense, sys.ops[OP_AIT], dT});
  KU[RES_P] = {{-1.0, sys.ops[OP_AEQ], &dX}, {1.0, sys.ops[OP_KY], &dY}};
  if (sys.ineq) KU[RES_T] = {{-sys.sense, sys.ops[OP_TA], &dX}, {1.0, sys.ops[OP_DK], dT}};
  KU[RES_C] = {{1.0, sys.ops[OP_LZ], &dX}, {1.0, sys.ops[OP_LX], &dZ}};
  // every pair's four-layer environment must stay within a memory budget;
  // otherwise the check is not made (res = rhs = -1)
  const double budget = 3.2e7;   // doubles (256 MiB) per environment
  for (int b = 0; b < 4; ++b) {
    std::vector<Img> all = KU[b];
    all.insert(all.end(), R[b].begin(), R[b].end());
    for (size_t i = 0; i < all.size(); ++i)
      for (size_t j = i; j < all.size(); ++j)
        for (int k = 0; k <= all[i].vec->d; ++k) {
          const double e = (double)all[i].vec->r[k] * (all[i].op ? all[i].op->r[k] : 1) *
                           (all[j].op ? all[j].op->r[k] : 1) * all[j].vec->r[k];
          if (e * 4.0 > budget) {
            *res = *rhs = -1.0;
            return;
          }
        }
  }
  // ||sum_i coef_i O_i v_i||^2 of every block row from the pairwise inner
  // products, all pairs of all rows in one batched evaluation; the pairs of
  // the right-hand-side terms alone (||R||) are a subset of them
  std::vector<OpDotPair> pairs;
  struct PairUse {
    int b;
    double w;    // weight in ||K dU + R||^2
    bool in_r;   // also a pair of ||R||^2
  };
  std::vector<PairUse> use;
  const bool cached = rr && rr->have;
  for (int b = 0; b < 4; ++b) {
    const int nk = (int)KU[b].size();
    std::vector<Img> all = KU[b];
    all.insert(all.end(), R[b].begin(), R[b].end());
    for (size_t i = 0; i < all.size(); ++i)
      for (size_t j = i; j < all.size(); ++j) {
        const bool in_r = (int)i >= nk && (int)j >= nk;
        if (in_r && cached) continue;   // ||R_b||^2 is known
        pairs.push_back({all[i].vec, all[i].op, all[j].vec, all[j].op});
        use.push_back({b, (i == j ? 1.0 : 2.0) * all[i].coef * all[j].coef, in_r});
      }
  }
  const std::vector<double> ip = tt_op_dots(pairs, c);
  double e2[4] = {0.0, 0.0, 0.0, 0.0}, r2[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t q = 0; q < ip.size(); ++q) {
    e2[use[q].b] += use[q].w * ip[q];
    if (use[q].in_r) r2[use[q].b] += use[q].w * ip[q];
  }
  if (cached) {
    for (int b = 0; b < 4; ++b) {
      r2[b] = rr->r2[b];
      e2[b] += r2[b];
    }
  } else if (rr) {
    for (int b = 0; b < 4; ++b) rr->r2[b] = r2[b];
    rr->have = true;
  }
  double es = 0.0, rs = 0.0;
  for (int b = 0; b < 4; ++b) {
    es += std::max(e2[b], 0.0);
    rs += std::max(r2[b], 0.0);
  }
  *res = std::sqrt(es);
  *rhs = std::sqrt(rs);
}

namespace {

// rows of block b (rho rows of len, taken from Eb[b]) scaled by 1 / ||Eb[b]||
// into out[b]; a zero block gives zero rows.  One workgroup per block.
__global__ __launch_bounds__(256) void normalize_blocks_kernel(const double* Eb, long blk, int rho, int len,
                                                               const int* which, bool transpose, double* out) {
  __shared__ double red[256];
  const double* y = Eb + (size_t)which[blockIdx.x] * blk;
  double* dst = out + (size_t)blockIdx.x * blk;
  double sq = 0.0;
  for (long t = threadIdx.x; t < blk; t += 256) sq += y[t] * y[t];
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
  // transpose: y is [len][rho] -> rows [rho][len]
  for (long t = threadIdx.x; t < blk; t += 256)
    dst[t] = sc * (transpose ? y[(t % len) * rho + t / len] : y[t]);
}

}  // namespace

namespace {

// Candidate enrichment rows at core k: every block row b of E = K dU + R
// (eq. (tt-kkt-newton-system), the current block core as dU_k) projected with
// the frame's environments behind the block and the sketch's ahead of it.
// dir > 0: E_b[a][i][t] (t: sketch rank) -> rows [t][(a,i)]; dir < 0:
// E_b[t][i][b] -> rows [t][(i,b)].  Each block row is scaled to unit norm so
// that every row of the system contributes.  Returns the number of rows.
int residual_candidates(const NewtonSys& sys, Envs& envs, Envs& sk, const BlockTT& W, int k, int dir,
                        const int* key_of_op, const std::vector<int>& key_of_term, int key_id, int rho, DevBuf& cand,
                        Ctx& c) {
  const int L = sys.L();
  const int r = W.r[k], s = W.r[k + 1];
  const long p = (long)r * 4 * s;
  struct Src {
    int row;
    double coef;
    int key;
    const double* x;
    int rc, rd;
  };
  std::vector<Src> src;
  auto comp = [&](int l) { return W.blk.get() + (size_t)l * p; };
  src.push_back({RES_D, 1.0, key_id, comp(L), r, s});
  src.push_back({RES_D, -1.0, key_of_op[OP_AEQT], comp(1), r, s});
  if (sys.ineq) src.push_back({RES_D, -sys.sense, key_of_op[OP_AIT], comp(2), r, s});
  src.push_back({RES_P, -1.0, key_of_op[OP_AEQ], comp(0), r, s});
  src.push_back({RES_P, 1.0, key_of_op[OP_KY], comp(1), r, s});
  if (sys.ineq) {
    src.push_back({RES_T, -sys.sense, key_of_op[OP_TA], comp(0), r, s});
    src.push_back({RES_T, 1.0, key_of_op[OP_DK], comp(2), r, s});
  }
  src.push_back({RES_C, 1.0, key_of_op[OP_LZ], comp(0), r, s});
  src.push_back({RES_C, 1.0, key_of_op[OP_LX], comp(L), r, s});
  for (size_t t = 0; t < sys.terms.size(); ++t) {
    const Term& tm = sys.terms[t];
    src.push_back({tm.res, tm.coef, key_of_term[t], tm.vec->core(k), tm.vec->r[k], tm.vec->r[k + 1]});
  }
  const int nrow = sys.ineq ? 4 : 3;
  const int rows_out = dir > 0 ? r * 4 : 4 * s;   // length of a candidate row
  const long blk = (long)rho * rows_out;           // one residual block row
  DevBuf Eb((size_t)4 * blk);
  fill(4 * blk, 0.0, Eb.get(), c.s);
  std::vector<DevBuf> operm(src.size());
  std::vector<LocalApplyArgs> v;
  for (size_t i = 0; i < src.size(); ++i) {
    const Src& q = src[i];
    TT_REQUIRE(q.key >= 0, "residual enrichment: missing environment");
    const EnvKey& e = envs.keys[q.key];
    const int R0 = envs.op_rank(e, k), R1 = envs.op_rank(e, k + 1);
    const double* Op = nullptr;
    if (e.op) {
      operm[i].reserve((size_t)e.op->core_size(k));
      permute_op_core(e.op->core(k), R0, 4, R1, operm[i].get(), c.s);
      Op = operm[i].get();
    }
    double* y = Eb.get() + (size_t)q.row * blk;
    if (dir > 0)   // [a][i][t]
      v.push_back({envs.L[q.key][k].get(), r, R0, q.rc, Op, 4, sk.R[q.key][k].get(), rho, R1, q.rd, q.x, y, q.coef,
                   1.0});
    else           // [t][i][b]
      v.push_back({sk.L[q.key][k].get(), rho, R0, q.rc, Op, 4, envs.R[q.key][k].get(), s, R1, q.rd, q.x, y, q.coef,
                   1.0});
  }
  local_apply_many(v, c);
  // rows of the candidates, one residual block row after another, each block
  // scaled to unit norm on the device (a zero block gives zero rows, which the
  // principal directions ignore)
  std::vector<int> used = {RES_D, RES_P};
  if (sys.ineq) used.push_back(RES_T);
  used.push_back(RES_C);
  c.ired.reserve(8);
  int* wd = reinterpret_cast<int*>(c.ired.get()) + 4;
  TT_HIP(hipMemcpyAsync(wd, used.data(), sizeof(int) * used.size(), hipMemcpyHostToDevice, c.s));
  cand.reserve((size_t)nrow * blk);
  hipLaunchKernelGGL(normalize_blocks_kernel, dim3((unsigned)used.size()), dim3(256), 0, c.s, Eb.get(), blk, rho,
                     rows_out, wd, dir > 0, cand.get());
  TT_HIP(hipGetLastError());
  c.sync();   // the host copy of `used` must be consumed before it goes out of scope
  return (int)used.size() * rho;
}

}  // namespace

void amen_solve(const NewtonSys& sys, BlockTT& W, const AmenParams& prm, AmenInfo& info, Ctx& c) {
  // The block sits at an end core: core 0 (the first sweep runs left to
  // right) or core d-1, where the previous solve's last sweep left it (the
  // first sweep runs right to left).  Either way every other core is
  // orthogonal towards the block, which is what the environments assume.
  const bool from_right = W.pos == W.d - 1 && W.d > 1;
  TT_REQUIRE(W.pos == 0 || from_right, "amen_solve expects the block at an end core");
  TT_REQUIRE(W.Lp == sys.Lp(), "block size");
  const int d = W.d;
  const int L = sys.L();
  // environment keys: system operators (trial = W), then residual terms
  std::vector<EnvKey> keys;
  int key_of_op[OP_COUNT];
  for (int o = 0; o < OP_COUNT; ++o) {
    key_of_op[o] = -1;
    if (!sys.ops[o]) continue;
    if (o >= OP_EXTRA0) continue;   // operators used only by residual terms
    key_of_op[o] = (int)keys.size();
    keys.push_back({sys.ops[o], nullptr});
  }
  std::vector<int> key_of_term(sys.terms.size());
  for (size_t t = 0; t < sys.terms.size(); ++t) {
    key_of_term[t] = (int)keys.size();
    keys.push_back({sys.terms[t].op >= 0 ? sys.ops[sys.terms[t].op] : nullptr, sys.terms[t].vec});
  }
  // residual enrichment (Sec. 2.3, AMEn of Dolgov and Savostyanov): the kick
  // directions at a block move are the leading directions of the Newton
  // residual E = K dU + R (unreduced block rows) projected on the frame's side
  // behind the block and on a seeded Gaussian TT sketch V of rank rho ahead of
  // it (reading: the sketch stands in for AMEn's rank-rho residual TT)
  const bool resid = prm.enrich == 1 && prm.kick > 0;
  int key_id = -1;
  if (resid) {
    key_id = (int)keys.size();
    keys.push_back({nullptr, nullptr});
  }
  Envs envs;
  envs.init(keys, d, c);
  const int rho = prm.kick + 2;
  TT V;
  Envs sk;
  if (resid) {
    V = TT(d, 4, 1);
    for (int k = 1; k < d; ++k) V.r[k] = rho;
    for (int k = 0; k < d; ++k) {
      V.alloc(k);
      random_block(V.core(k), V.core_size(k), prm.seed * 7919ull + 104729ull * (unsigned long long)k + 17ull, c);
    }
    sk.test = &V;
    sk.init(keys, d, c);
  }
  double t0 = now();
  if (from_right)
    for (int k = 0; k < d - 1; ++k) envs.update_left(W, k, c);
  else
    for (int k = d - 1; k > 0; --k) envs.update_right(W, k, c);
  c.sync();
  info.t_env += now() - t0;
  const double tol_svd = prm.tol / std::sqrt((double)d);
  int dir = from_right ? -1 : +1;
  info.sweeps = 0;
  info.krylov_iters = 0;
  DevBuf Rall;                  // the four projected residuals, contiguous (one fill)
  double* Rhat_p[4] = {nullptr, nullptr, nullptr, nullptr};
  DevBuf f, u, Ku, dz;
  std::vector<int> bj_ref(d, 0);   // block-Jacobi Krylov counts per core (MLP fallback budget)
  std::vector<double> res_hist;   // max_res of each sweep
  std::vector<double> glob_hist;  // global Newton residual ratio of each half-sweep (-1: not evaluated)
  // The global rule pays one residual evaluation per half-sweep: it is used
  // only while that is cheap next to a half-sweep, i.e. while the four-layer
  // environments of the operator-image products stay small (frame rank r,
  // operator ranks R: r^2 R^2 per core below 2^20 doubles; at r = 32, R = 64
  // one evaluation cost as much as a quarter of the iteration).
  bool glob_cheap = true;
  ResidualRhs rhs_cache;   // ||R||^2 of the block rows, the same for every half-sweep
  {
    size_t rmax = 1, Rmax = 1;
    for (int x : W.r) rmax = std::max(rmax, (size_t)std::max(x, 1));
    rmax = std::max(rmax, (size_t)prm.rank_cap);
    for (const TT* op : sys.ops)
      if (op) Rmax = std::max(Rmax, (size_t)op->max_rank());
    glob_cheap = rmax * rmax * Rmax * Rmax <= (size_t(1) << 20);
  }
  for (int sweep = 0; sweep < prm.max_sweeps; ++sweep) {
    double max_res = 0.0;
    info.newton_res_final = false;   // the direction changes in this half-sweep
    const bool enrich_now = resid && sweep < prm.kick_sweeps;
    // sketch environments on the side ahead of the block (its frame cores
    // stay fixed until the sweep reaches them), built at the first request
    // for candidates in this half-sweep (core k0): the side ahead of k0 is
    // all that this and every later request of the half-sweep reads
    bool sk_fresh = false;
    auto ensure_sketch = [&](int k0) {
      if (sk_fresh) return;
      const double te = now();
      if (dir > 0)
        for (int k = d - 1; k > k0; --k) sk.update_right(W, k, c);
      else
        for (int k = 0; k < k0; ++k) sk.update_left(W, k, c);
      c.sync();
      info.t_env += now() - te;
      sk_fresh = true;
    };
    for (int step = 0; step < d; ++step) {
      const int k = (dir > 0) ? step : d - 1 - step;
      TT_REQUIRE(W.pos == k, "block position");
      LocalKKT K;
      K.sys = &sys;
      K.envs = &envs;
      K.W = &W;
      K.k = k;
      for (int o = 0; o < OP_COUNT; ++o) K.key_of_op[o] = key_of_op[o];
      K.setup(c);
      const int p = K.p, r = K.r, s = K.s;
      const long n = (long)L * p;
      // projected residuals
      Rall.reserve((size_t)4 * p);
      fill(4L * p, 0.0, Rall.get(), c.s);
      for (int q = 0; q < 4; ++q) Rhat_p[q] = Rall.get() + (size_t)q * p;
      // the terms' projections in grouped stage launches (terms of one block
      // residual keep their order)
      // a term's operator is one of the system's (already permuted by
      // K.setup) or a further one, permuted here (all in one launch)
      std::vector<DevBuf> operms(sys.terms.size());
      std::vector<LocalApplyArgs> proj;
      std::vector<const double*> term_op(sys.terms.size(), nullptr);
      {
        std::vector<PermJob> jobs;
        for (size_t t = 0; t < sys.terms.size(); ++t) {
          const EnvKey& e = envs.keys[key_of_term[t]];
          if (!e.op) continue;
          for (int o = 0; o < OP_COUNT && !term_op[t]; ++o)
            if (K.key_of_op[o] >= 0 && sys.ops[o] == e.op) term_op[t] = K.operm[o].get();
          if (term_op[t]) continue;
          operms[t].reserve((size_t)e.op->core_size(k));
          jobs.push_back({e.op->core(k), operms[t].get(), {envs.op_rank(e, k), 4, 4, envs.op_rank(e, k + 1)},
                          {1, 3, 0, 2}});
          term_op[t] = operms[t].get();
        }
        permute_many(jobs, c.s);
      }
      for (size_t t = 0; t < sys.terms.size(); ++t) {
        const Term& tm = sys.terms[t];
        const int key = key_of_term[t];
        const EnvKey& e = envs.keys[key];
        const int R0 = envs.op_rank(e, k), R1 = envs.op_rank(e, k + 1);
        const int rc = e.trial->r[k], rd = e.trial->r[k + 1];
        const double* Op = e.op ? term_op[t] : nullptr;
        proj.push_back({envs.L[key][k].get(), r, R0, rc, Op, 4, envs.R[key][k].get(), s, R1, rd, e.trial->core(k),
                        Rhat_p[tm.res], tm.coef, 1.0});
      }
      local_apply_many(proj, c);   // the permuted cores are recycled in stream order
      // local right-hand side f = [-Rp; (-Rt;) -Rc + LX^ Rd]
      f.reserve(n);
      axpby(p, -1.0, Rhat_p[RES_P], 0.0, f.get(), c.s);
      if (sys.ineq) axpby(p, -1.0, Rhat_p[RES_T], 0.0, f.get() + p, c.s);
      double* fc = f.get() + (size_t)(L - 1) * p;
      K.apply(OP_LX, Rhat_p[RES_D], fc, 1.0, 0.0, c);
      axpby(p, -1.0, Rhat_p[RES_C], 1.0, fc, c.s);
      // initial guess: current block components
      u.reserve(n);
      TT_HIP(hipMemcpyAsync(u.get(), W.blk.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
      Ku.reserve(n);
      K.matvec(u.get(), Ku.get(), c);
      axpby(n, 1.0, f.get(), -1.0, Ku.get(), c.s);
      const double fn = dev_norm(f.get(), n, c);
      const double res0 = dev_norm(Ku.get(), n, c) / (fn > 0 ? fn : 1.0);
      max_res = std::max(max_res, res0);
      if (prm.mlp && prm.collect_probes > 0 && prm.mlp->ds_N < prm.collect_cap && fn > 0.0) {
        // the local systems the solver emits, as training data of the learned preconditioner
        BlockJacobi raw, inv;
        build_block_jacobi(K, raw, c);
        inv.copy_from(raw, c);
        inv.invert(c);
        float ctx[4];
        mlp_context(K, prm, ctx);
        FBuf F, Rr, Y, S, Wt;
        mlp_block_data(raw, inv, [&](const double* x, double* y) { K.matvec(x, y, c); }, ctx, prm.collect_probes,
                       prm.seed * 7ull + (unsigned long long)(sweep * 131 + k), F, Rr, Y, S, Wt, c);
        const MlpBatch mb{K.r * K.s, prm.collect_probes, L * 4, F.get(), Rr.get(), Y.get(), S.get(), Wt.get()};
        if (prm.mlp->out == mb.n * mb.n) prm.mlp->append(mb, prm.collect_cap, c);
      }
      double ts = now();
      if (fn == 0.0) {
        fill(n, 0.0, u.get(), c.s);
      } else if (n <= prm.direct_max) {
        // the paper's block elimination; LU of the whole block system when
        // inequalities are present or L_Z^ is numerically singular
        const bool ok = !sys.ineq && solve_elim(K, Rhat_p[RES_D], Rhat_p[RES_P], Rhat_p[RES_C], u.get(), c);
        if (!ok) solve_direct(K, f.get(), u.get(), c);
      } else {
        double rel = 0.0;
        int its = solve_gmres(K, f.get(), u.get(), prm, bj_ref, info, &rel, c);
        info.krylov_iters += its;
      }
      // dZ_k = Aeq^T^ y (+ s Aineq^T^ t) - R_d^
      dz.reserve(p);
      K.apply(OP_AEQT, u.get() + p, K.tmp.get(), 1.0, 0.0, c);
      if (sys.ineq) K.apply(OP_AIT, u.get() + 2 * p, K.tmp.get(), sys.sense, 1.0, c);
      // write the block core [x, y, (t), dz]
      W.blk.reserve((size_t)(L + 1) * p);
      TT_HIP(hipMemcpyAsync(W.blk.get(), u.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
      hipLaunchKernelGGL(stack_dz_kernel, dim3(nblocks(p, 256)), dim3(256), 0, c.s, W.blk.get() + n, K.tmp.get(),
                         Rhat_p[RES_D], (long)p);
      TT_HIP(hipGetLastError());
      info.t_solve += now() - ts;   // the block core's last kernels finish under the split
      // sketched residual of the local system: candidate enrichment rows,
      // computed by the split only when the cap leaves room for them
      DevBuf cand;
      const CandidateFn cand_fn = [&](const double** rows) {
        ensure_sketch(k);
        const int nc = residual_candidates(sys, envs, sk, W, k, dir, key_of_op, key_of_term, key_id, rho, cand, c);
        *rows = cand.get();
        return nc;
      };
      const CandidateFn* cand_use =
          (enrich_now && ((dir > 0 && k < d - 1) || (dir < 0 && k > 0))) ? &cand_fn : nullptr;
      // move the block index and extend the environments
      if (dir > 0 && k < d - 1) {
        double t1 = now();
        info.capped |= split_block(W, +1, tol_svd, prm.rank_cap, c, sweep < prm.kick_sweeps ? prm.kick : 0,
                    prm.seed * 1000003ull + (unsigned long long)(sweep * 131 + k), cand_use);
        info.t_svd += now() - t1;
        t1 = now();
        envs.update_left(W, k, c);   // its kernels finish under the next local solve
        info.t_env += now() - t1;
      } else if (dir < 0 && k > 0) {
        double t1 = now();
        info.capped |= split_block(W, -1, tol_svd, prm.rank_cap, c, sweep < prm.kick_sweeps ? prm.kick : 0,
                    prm.seed * 1000003ull + (unsigned long long)(sweep * 131 + k) + 7777ull, cand_use);
        info.t_svd += now() - t1;
        t1 = now();
        envs.update_right(W, k, c);   // its kernels finish under the next local solve
        info.t_env += now() - t1;
      }
    }
    info.sweeps += 1;
    info.last_max_res = max_res;
    if (prm.verbose >= 2) {
      std::fprintf(stderr, "    amen sweep %d dir %+d max_res %.3e tol %.3e ranks", sweep, dir, max_res, prm.tol);
      for (int x : W.r) std::fprintf(stderr, " %d", x);
      std::fprintf(stderr, "\n");
    }
    dir = -dir;
    if (max_res < prm.tol && sweep >= 1) break;
    // With the rank cap binding the sweeps settle into a cycle of period two
    // (the same truncated frames in each direction) above the target: stop
    // once a sweep improves on the one two back (same direction) by less
    // than 10 %.
    res_hist.push_back(max_res);
    if (info.capped && sweep >= 2 && max_res > 0.9 * res_hist[sweep - 2]) break;
    // Capped solves, measured globally: once the cap binds, further
    // half-sweeps mostly cycle between truncated frames.  After every
    // half-sweep of such a solve the FP64 residual ||K dU + R|| / ||R|| of
    // the whole Newton system is evaluated (batched operator-image inner
    // products); the solve stops when it meets the forcing bound eta = 2 tol
    // (Lemma "AMEn Directions as Inexact Newton Directions"), or when it is
    // below 1 and improves on the half-sweep two back (same direction) by
    // less than 10 %.
    if (prm.global_stop && info.capped && glob_cheap) {
      const double tg = now();
      double res = 0.0, rhs = 0.0;
      newton_residual(sys, W, &res, &rhs, c, &rhs_cache);
      info.t_check += now() - tg;
      if (res >= 0.0 && rhs > 0.0) {
        const double ratio = res / rhs;
        glob_hist.resize(sweep + 1, -1.0);
        glob_hist[sweep] = ratio;
        info.newton_res = ratio;
        info.newton_res_final = true;
        const bool met = ratio <= 2.0 * prm.tol;
        const bool flat = sweep >= 2 && glob_hist[sweep - 2] >= 0.0 && ratio < 1.0 &&
                          ratio > 0.9 * glob_hist[sweep - 2];
        if (met || flat) break;
      }
    }
  }
  // The block stays where the last sweep left it (an end core): moving it back
  // without truncation would only merge the components into the shared frame
  // and inflate every component's TT ranks (up to L+1 times the frame rank).
  info.max_rank = 0;
  for (int x : W.r) info.max_rank = std::max(info.max_rank, x);
}

}  // namespace ttipm
