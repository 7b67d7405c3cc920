// The C ABI (include/ttipm.h): argument checks, marshalling of tt_view
// structures into device TTs, and translation of internal errors into status
// codes.  No C++ exception crosses this boundary.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>

#include "../../include/ttipm.h"
#include "amen.hpp"
#include "blocked.hpp"
#include "krylov.hpp"
#include "mlp.hpp"
#include "noalloc.hpp"
#include "dense.hpp"
#include "ipm.hpp"
#include "ttops.hpp"

namespace ttipm {
const char* last_error();
}

using namespace ttipm;

struct ttipm_problem {
  Problem P;
};

struct ttipm_state {
  State S;
  int d = 0;
};

namespace {

std::mutex g_ctx_mu;
std::map<void*, std::unique_ptr<Ctx>> g_ctx;

// One execution context (scratch buffers) per stream.
Ctx& ctx_for(void* stream) {
  std::lock_guard<std::mutex> g(g_ctx_mu);
  auto it = g_ctx.find(stream);
  if (it != g_ctx.end()) return *it->second;
  auto c = std::make_unique<Ctx>();
  c->s = as_stream(stream);
  Ctx& ref = *c;
  g_ctx[stream] = std::move(c);
  return ref;
}

template <typename F>
int guarded(F&& f) {
  try {
    set_last_error("");
    return f();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return TT_ERR_ARG;
  } catch (...) {
    set_last_error("unknown error");
    return TT_ERR_ARG;
  }
}

void check_view(const tt_view* v, const char* name) {
  if (!v) throw Error(TT_ERR_ARG, std::string(name) + " is NULL");
  if (v->d < 1 || !v->ranks || !v->cores) throw Error(TT_ERR_ARG, std::string(name) + ": empty view");
  if (v->dtype != TT_F64) throw Error(TT_ERR_ARG, std::string(name) + ": only TT_F64 views are accepted");
  if (v->ranks[0] != 1 || v->ranks[v->d] != 1) throw Error(TT_ERR_ARG, std::string(name) + ": boundary ranks must be 1");
  if (v->m_out < 1 || v->m_in < 1) throw Error(TT_ERR_ARG, std::string(name) + ": mode sizes");
  for (int k = 0; k < v->d; ++k) {
    if (v->ranks[k + 1] < 1) throw Error(TT_ERR_ARG, std::string(name) + ": ranks must be positive");
    if (v->capacity_rank > 0 && v->ranks[k + 1] > v->capacity_rank)
      throw Error(TT_ERR_ARG, std::string(name) + ": a rank exceeds capacity_rank");
    if (!v->cores[k]) throw Error(TT_ERR_ARG, std::string(name) + ": NULL core pointer");
  }
}

// Non-owning TT over caller buffers (shallow): copies are made only where the
// library needs its own storage.
TT view_as_tt(const tt_view& v, Ctx& c) { return tt_from_view(v, c); }

}  // namespace

extern "C" {

const char* tt_last_error(void) { return ttipm::last_error(); }

const char* tt_version(void) { return "ttipm-mi355x 0.1 (gfx950)"; }

int tt_abi_sizes(size_t* out, int32_t n) {
  const size_t sz[] = {sizeof(tt_view),         sizeof(tt_proj_op),     sizeof(tt_local_block),
                       sizeof(tt_local_op),     sizeof(tt_solve_params), sizeof(tt_solve_info),
                       sizeof(ttipm_problem_desc), sizeof(tt_mlp_batch), sizeof(tt_kernel_stat),
                       sizeof(ttipm_params),    sizeof(ttipm_step_info), sizeof(ttipm_result)};
  const int count = (int)(sizeof(sz) / sizeof(sz[0]));
  for (int i = 0; out && i < n && i < count; ++i) out[i] = sz[i];
  return count;
}

int tt_profile_start(int32_t period) {
  return guarded([&]() -> int {
    if (period < 1) throw Error(TT_ERR_ARG, "period must be >= 1");
    prof_start(period);
    return TT_OK;
  });
}

int tt_profile_stop(tt_kernel_stat* out, int32_t cap, int32_t* count) {
  return guarded([&]() -> int {
    if (cap > 0 && !out) throw Error(TT_ERR_ARG, "out is NULL");
    const int n = prof_stop(out, cap < 0 ? 0 : cap);
    if (count) *count = n;
    return TT_OK;
  });
}

int tt_contract_interfaces(const tt_view* test, const tt_view* op, const tt_view* trial, int32_t k, int32_t dir,
                           const double* phi_in, double* phi_out, void* stream) {
  return guarded([&]() -> int {
    check_view(test, "test");
    check_view(trial, "trial");
    if (op) check_view(op, "op");
    if (test->m_in != 1 || trial->m_in != 1) throw Error(TT_ERR_ARG, "test and trial must be TT vectors");
    if (test->d != trial->d || (op && op->d != test->d)) throw Error(TT_ERR_ARG, "d mismatch");
    if (k < 0 || k >= test->d) throw Error(TT_ERR_ARG, "core index out of range");
    if (!phi_in || !phi_out) throw Error(TT_ERR_ARG, "NULL environment pointer");
    if (op && (op->m_out != test->m_out || op->m_in != trial->m_out))
      throw Error(TT_ERR_ARG, "operator modes must be test.m_out x trial.m_out");
    if (!op && test->m_out != trial->m_out) throw Error(TT_ERR_ARG, "identity needs equal mode sizes");
    Ctx& c = ctx_for(stream);
    c.prec = GemmPrec::F64;
    const int ra = test->ranks[k], ra2 = test->ranks[k + 1];
    const int rc = trial->ranks[k], rc2 = trial->ranks[k + 1];
    const int R0 = op ? op->ranks[k] : 1, R1 = op ? op->ranks[k + 1] : 1;
    const int mo = test->m_out, mi = trial->m_out;
    if (dir == TT_LEFT)
      env_left_step(phi_in, ra, R0, rc, test->cores[k], mo, ra2, op ? op->cores[k] : nullptr, R1, mi, trial->cores[k],
                    rc2, phi_out, c);
    else if (dir == TT_RIGHT)
      env_right_step(phi_in, ra2, R1, rc2, test->cores[k], mo, ra, op ? op->cores[k] : nullptr, R0, mi,
                     trial->cores[k], rc, phi_out, c);
    else
      throw Error(TT_ERR_ARG, "dir must be TT_LEFT or TT_RIGHT");
    return TT_OK;
  });
}

namespace {

void check_local_op(const tt_local_op* K) {
  if (!K || K->r < 1 || K->rp < 1 || K->m < 1 || K->L < 1 || K->nblocks < 0 || (K->nblocks && !K->blocks))
    throw Error(TT_ERR_ARG, "invalid tt_local_op");
  if (K->precision != TTIPM_F64 && K->precision != TTIPM_MIXED) throw Error(TT_ERR_ARG, "tt_local_op precision");
  for (int b = 0; b < K->nblocks; ++b) {
    const tt_local_block& B = K->blocks[b];
    if (B.row < 0 || B.row >= K->L || B.col < 0 || B.col >= K->L) throw Error(TT_ERR_ARG, "block position");
    if (B.nchain < 1 || B.nchain > 2) throw Error(TT_ERR_ARG, "nchain must be 1 or 2");
    for (int q = 0; q < B.nchain; ++q) {
      const tt_proj_op& o = B.op[q];
      if (!o.phiL || !o.phiR || o.R < 1 || o.Rp < 1) throw Error(TT_ERR_ARG, "projected operator");
      if (!o.core && (o.R != 1 || o.Rp != 1)) throw Error(TT_ERR_ARG, "identity operator needs R = Rp = 1");
    }
  }
}

// y = K x for the generic block description (chains of projected operators).
// The blocks' projected products in grouped stage launches: first operators
// of every block, then the second operators of the chained blocks; the
// products of one block row keep the block order within each level.
// y = K x.  With arena, the permuted cores, chain buffers, stage buffers and
// split-K partials come from it; with dry as well nothing is launched and
// arena->used / *ws_need receive the scratch the call needs (a dry run takes
// an arena whose base is a placeholder address: its pointers are compared,
// never dereferenced, so the launch grouping is that of the real call).
void generic_matvec(const tt_local_op* K, const double* x, double* y, Ctx& c, Arena* arena = nullptr,
                    bool dry = false, size_t* ws_need = nullptr) {
  const long p = (long)K->r * K->m * K->rp;
  if (!dry) fill((long)K->L * p, 0.0, y, c.s);
  // context-owned permuted cores and chain buffers: no allocation is released
  // while kernels may still use it
  size_t nb = 0;
  auto buf = [&](size_t n) {
    if (arena) return arena->take(n);
    if (c.lbuf.size() <= nb) c.lbuf.resize(nb + 1);
    c.lbuf[nb].reserve(n);
    return c.lbuf[nb++].get();
  };
  auto args = [&](const tt_proj_op& o, const double* xin, double* yout, double alpha, double beta) {
    double* perm = nullptr;
    if (o.core) {
      perm = buf((size_t)o.R * K->m * K->m * o.Rp);
      if (!dry) permute_op_core(o.core, o.R, K->m, o.Rp, perm, c.s);
    }
    return LocalApplyArgs{o.phiL, K->r, o.R, K->r, perm, K->m, o.phiR, K->rp, o.Rp, K->rp, xin, yout, alpha, beta};
  };
  std::vector<LocalApplyArgs> lv0, lv1;
  for (int b = 0; b < K->nblocks; ++b) {
    const tt_local_block& B = K->blocks[b];
    const double* xin = x + (long)B.col * p;
    double* yout = y + (long)B.row * p;
    if (B.nchain == 1) {
      lv0.push_back(args(B.op[0], xin, yout, B.coeff, 1.0));
    } else {
      double* tb = buf((size_t)p);
      lv0.push_back(args(B.op[0], xin, tb, 1.0, 0.0));
      lv1.push_back(args(B.op[1], tb, yout, B.coeff, 1.0));
    }
  }
  // the two levels run one after the other on the stream; with an arena the
  // second level's stage buffers follow the first level's
  local_apply_many(lv0, c, arena, dry, ws_need);
  local_apply_many(lv1, c, arena, dry, ws_need);
}

}  // namespace

int tt_local_matvec(const tt_local_op* K, const double* x, double* y, void* stream) {
  return guarded([&]() -> int {
    check_local_op(K);
    if (!x || !y) throw Error(TT_ERR_ARG, "NULL vector");
    Ctx& c = ctx_for(stream);
    c.prec = K->precision == TTIPM_MIXED ? GemmPrec::BF16 : GemmPrec::F64;
    generic_matvec(K, x, y, c);
    c.prec = GemmPrec::F64;
    return TT_OK;
  });
}

int tt_local_matvec_noalloc(const tt_local_op* K, const double* x, double* y, void* stream) {
  return guarded([&]() -> int {
    check_local_op(K);
    if (!x || !y) throw Error(TT_ERR_ARG, "NULL vector");
    size_t cap = 0;
    double* scratch = noalloc_scratch(&cap);
    // a context of the caller's stream that never reserves memory: every
    // buffer of the call comes from the static scratch array
    Ctx c;
    c.s = as_stream(stream);
    c.prec = K->precision == TTIPM_MIXED ? GemmPrec::BF16 : GemmPrec::F64;
    Arena plan;
    plan.base = reinterpret_cast<double*>(uintptr_t(1) << 20);   // placeholder, never dereferenced
    plan.cap = size_t(1) << 56;
    size_t ws_need = 0;
    generic_matvec(K, x, y, c, &plan, true, &ws_need);
    const size_t need = ((plan.used + 31) & ~size_t(31)) + ws_need;
    if (need > cap) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "tt_local_matvec_noalloc: the call needs %.1f MiB of scratch, the limit is %.1f MiB",
                    need * 8.0 / (1 << 20), cap * 8.0 / (1 << 20));
      throw Error(TT_ERR_ARG, msg);
    }
    Arena run;
    run.base = scratch;
    run.cap = cap;
    generic_matvec(K, x, y, c, &run, false, nullptr);
    return TT_OK;
  });
}

int tt_local_solve(const tt_local_op* K, const double* rhs, double* x, const tt_solve_params* p, tt_solve_info* info,
                   void* stream) {
  return guarded([&]() -> int {
    check_local_op(K);
    if (!rhs || !x || !p) throw Error(TT_ERR_ARG, "NULL argument");
    if (rhs == x) throw Error(TT_ERR_ARG, "rhs and x must not alias");
    if (p->method < TT_SOLVE_AUTO || p->method > TT_SOLVE_CHOLESKY) throw Error(TT_ERR_ARG, "unknown solve method");
    Ctx& c = ctx_for(stream);
    c.prec = GemmPrec::F64;
    const long n = (long)K->L * K->r * K->m * K->rp;
    tt_solve_info inf{};
    int method = p->method;
    if (method == TT_SOLVE_AUTO) method = (n <= p->direct_max) ? TT_SOLVE_DIRECT : TT_SOLVE_GMRES;
    if (method == TT_SOLVE_DIRECT || method == TT_SOLVE_CHOLESKY) {
      // dense K by applying the operator to unit vectors, then a blocked factorisation
      if (n > 8192) throw Error(TT_ERR_ARG, "direct solve limited to 8192 unknowns");
      DevBuf Kd((size_t)n * n), e(n), Kt((size_t)n * n);
      for (long j = 0; j < n; ++j) {
        fill(n, 0.0, e.get(), c.s);
        fill(1, 1.0, e.get() + j, c.s);
        generic_matvec(K, e.get(), Kt.get() + (size_t)j * n, c);   // column j (stored as row j of Kt)
      }
      permute(Kt.get(), Kd.get(), {n, n}, {1, 0}, c.s);
      TT_HIP(hipMemcpyAsync(x, rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
      BlockedFactors f;
      if (method == TT_SOLVE_CHOLESKY) {
        dense_symmetrize(Kd.get(), (int)n, c.s);
        if (chol_blocked(Kd.get(), (int)n, f, c)) throw Error(TT_ERR_NUMERIC, "local system not positive definite");
        trsm_blocked(Kd.get(), (int)n, f, x, 1, false, c);
        trsm_blocked(Kd.get(), (int)n, f, x, 1, true, c);
      } else {
        if (lu_blocked(Kd.get(), (int)n, f, c)) throw Error(TT_ERR_NUMERIC, "singular local system");
        lu_solve_blocked(Kd.get(), (int)n, f, x, 1, c);
      }
      c.sync();
      inf.method_used = method;
      inf.iters = 0;
    } else {
      // restarted GMRES (CGS2), right-preconditioned; mixed: BF16 Arnoldi products, FP64 refinement
      const bool mixed = p->precision == TTIPM_MIXED;
      BlockJacobi bj;
      KrylovOps ops;
      ops.matvec = [&](const double* xv, double* yv, bool low) {
        c.prec = low ? GemmPrec::BF16 : GemmPrec::F64;
        generic_matvec(K, xv, yv, c);
        c.prec = GemmPrec::F64;
      };
      inf.precond_used = TT_PREC_NONE;
      KrylovParams kp;
      kp.rtol = p->rtol;
      kp.restart = std::max(1, p->restart);
      kp.maxit = std::max(0, p->maxit);
      kp.mixed = mixed;
      KrylovInfo ki;
      if (p->precond == TT_PREC_BJACOBI || p->precond == TT_PREC_MLP) {
        if (p->precond == TT_PREC_MLP && !p->mlp) throw Error(TT_ERR_ARG, "TT_PREC_MLP needs an mlp handle");
        BlockJacobi raw;
        raw.init(K->r, K->rp, K->m, K->L, c);
        for (int b = 0; b < K->nblocks; ++b) {
          const tt_local_block& B = K->blocks[b];
          BlockJacobi::Op ch[2];
          for (int q = 0; q < B.nchain; ++q) ch[q] = {B.op[q].phiL, B.op[q].core, B.op[q].phiR, B.op[q].R, B.op[q].Rp};
          raw.add(B.row, B.col, B.coeff, ch, B.nchain, c);
        }
        bj.copy_from(raw, c);
        bj.invert(c);
        ops.precond = [&](const double* xv, double* yv) { bj.apply(xv, yv, c); };
        if (p->precond == TT_PREC_MLP) {
          // Fallback rule: the MLP preconditioner is kept only if it needs no
          // more Krylov iterations and reaches no worse a residual than block
          // Jacobi from the same initial guess.
          DevBuf x0(n), xb(n);
          TT_HIP(hipMemcpyAsync(x0.get(), x, sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
          TT_HIP(hipMemcpyAsync(xb.get(), x, sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
          KrylovInfo kb;
          gmres_solve(n, ops, rhs, xb.get(), kp, kb, c);
          BlockJacobi ml;
          ml.copy_from(bj, c);
          mlp_correct_blocks(const_cast<tt_mlp*>(static_cast<const tt_mlp*>(p->mlp))->net, raw, ml, p->context, c);
          KrylovOps mops = ops;
          mops.precond = [&](const double* xv, double* yv) { ml.apply(xv, yv, c); };
          gmres_solve(n, mops, rhs, x, kp, ki, c);
          const bool mlp_ok = ki.iters <= kb.iters && ki.rel_res <= std::max(kb.rel_res, p->rtol);
          if (mlp_ok) {
            inf.precond_used = TT_PREC_MLP;
          } else {
            TT_HIP(hipMemcpyAsync(x, xb.get(), sizeof(double) * n, hipMemcpyDeviceToDevice, c.s));
            ki = kb;
            inf.precond_used = TT_PREC_BJACOBI;
          }
          c.sync();
        } else {
          gmres_solve(n, ops, rhs, x, kp, ki, c);
          inf.precond_used = TT_PREC_BJACOBI;
        }
      } else {
        gmres_solve(n, ops, rhs, x, kp, ki, c);
      }
      inf.method_used = TT_SOLVE_GMRES;
      inf.iters = ki.iters;
      inf.rel_res = ki.rel_res;
    }
    // true residual in FP64
    if (inf.method_used != TT_SOLVE_GMRES) {
      DevBuf r0(n);
      generic_matvec(K, x, r0.get(), c);
      axpby(n, 1.0, rhs, -1.0, r0.get(), c.s);
      const double bn = dev_norm(rhs, n, c);
      inf.rel_res = bn > 0 ? dev_norm(r0.get(), n, c) / bn : 0.0;
    }
    if (info) *info = inf;
    c.sync();
    return (inf.rel_res <= p->rtol || inf.method_used != TT_SOLVE_GMRES) ? TT_OK : TT_ERR_NOT_CONVERGED;
  });
}

int tt_op_inner(const tt_view* vi, const tt_view* Oi, const tt_view* vj, const tt_view* Oj, double* out,
                void* stream) {
  return guarded([&]() -> int {
    check_view(vi, "vi");
    check_view(vj, "vj");
    if (!out) throw Error(TT_ERR_ARG, "NULL out");
    if (vi->m_in != 1 || vj->m_in != 1 || vi->m_out != vj->m_out || vi->d != vj->d)
      throw Error(TT_ERR_ARG, "vi and vj must be TT vectors with the same modes");
    for (const tt_view* O : {Oi, Oj}) {
      if (!O) continue;
      check_view(O, "operator");
      if (O->d != vi->d || O->m_out != vi->m_out || O->m_in != vi->m_out)
        throw Error(TT_ERR_ARG, "operator modes must match the vectors");
    }
    Ctx& c = ctx_for(stream);
    c.prec = GemmPrec::F64;
    TT a = tt_from_view(*vi, c), b = tt_from_view(*vj, c);
    std::unique_ptr<TT> A, B;
    if (Oi) A = std::make_unique<TT>(tt_from_view(*Oi, c));
    if (Oj) B = std::make_unique<TT>(tt_from_view(*Oj, c));
    *out = tt_op_dot(a, A.get(), b, B.get(), c);
    return TT_OK;
  });
}

int tt_round_workspace(const tt_view* t, size_t* bytes) {
  return guarded([&]() -> int {
    check_view(t, "t");
    if (!bytes) throw Error(TT_ERR_ARG, "NULL bytes");
    // bound on the device memory one rounding takes: the working copy and the
    // orthogonalised cores, then per bond the QR / one-sided Jacobi SVD
    // temporaries of the (r_k m) x r_{k+1} unfolding and the next core
    const double m = (double)t->m_out * t->m_in;
    double sum = 0.0, per_bond = 0.0;
    for (int k = 0; k < t->d; ++k) {
      const double rows = t->ranks[k] * m, cols = t->ranks[k + 1];
      sum += rows * cols;
      const double next = k + 1 < t->d ? cols * m * t->ranks[k + 2] : 0.0;
      per_bond = std::max(per_bond, 12.0 * rows * cols + 6.0 * cols * cols + 3.0 * next + 64.0 * cols);
    }
    *bytes = (size_t)(2.0 * 8.0 * (2.0 * sum + per_bond)) + ((size_t)1 << 20);
    return TT_OK;
  });
}

int tt_round(tt_view* t, double tol, int32_t tol_mode, int32_t max_rank, double* zeta_out, void* ws,
             size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    check_view(t, "t");
    if (!(tol >= 0.0)) throw Error(TT_ERR_ARG, "tol must be >= 0");
    if (max_rank < 1) throw Error(TT_ERR_ARG, "max_rank must be >= 1");
    if (ws && ((uintptr_t)ws & 255)) throw Error(TT_ERR_ARG, "workspace must be 256-byte aligned");
    auto run = [&](Ctx& c) {
      TT w = tt_from_view(*t, c);
      double eps = tol;
      if (tol_mode == TT_TOL_REL) eps = tol * tt_norm(w, c);
      bool capped = false;
      const double zeta = tt_round_abs(w, eps, max_rank, c, &capped);
      c.sync();
      // the caller's cores change only once the rounding has succeeded
      for (int k = 0; k < t->d; ++k)
        TT_HIP(hipMemcpyAsync(t->cores[k], w.core(k), sizeof(double) * w.core_size(k), hipMemcpyDeviceToDevice, c.s));
      for (int k = 0; k <= t->d; ++k) t->ranks[k] = w.r[k];
      c.sync();
      if (zeta_out) *zeta_out = zeta;
      return capped ? (int)TT_ERR_RANK_CAP : (int)TT_OK;
    };
    if (!ws) {
      Ctx& c = ctx_for(stream);
      c.prec = GemmPrec::F64;
      return run(c);
    }
    // every device buffer of the call comes from the caller's workspace: a
    // context of its own (destroyed, with its buffers, inside the scope)
    ArenaScope scope(ws, ws_bytes);
    Ctx c;
    c.s = as_stream(stream);
    c.prec = GemmPrec::F64;
    try {
      return run(c);
    } catch (...) {
      (void)hipStreamSynchronize(c.s);
      throw;
    }
  });
}

void ttipm_params_default(ttipm_params* p) {
  if (!p) return;
  p->eps_gap = 1e-4;
  p->stop_gap = 1e-4;
  p->eta0 = 1e-3;
  p->delta = 1e-4;
  p->cmu = 2.0;
  p->tau = 0.95;
  p->n_xz = 3;
  p->max_iter = 60;
  p->rank_cap = 16;
  p->iter_rank_cap = 0;
  p->amen_sweeps = 6;
  p->direct_max = 1024;
  p->gmres_restart = 40;
  p->gmres_maxit = 400;
  p->precision = TTIPM_F64;
  p->precond = TT_PREC_NONE;
  p->mlp = nullptr;
  p->eig_rank = 6;
  p->eig_sweeps = 2;
  p->verbose = 0;
  p->kick = 2;
  p->seed = 12345;
  p->kick_sweeps = 1 << 30;
  p->collect_probes = 0;
  p->collect_cap = 1 << 20;
  p->xz_fallback = 0;
  p->eig_kick = 2;
  p->g4_window = 4;
  p->g4_retries = 3;
  p->shift_mode = 1;
  p->newton_check = 1;
  p->refine_sweeps = 2;
  p->enrich = 1;
  p->combine_multipliers = 1;
  p->amen_global_stop = 1;
  p->finish = 0;
  p->finish_abs = 1e-3;
  p->finish_nu_max = 1e-3;
}

int ttipm_problem_create(const ttipm_problem_desc* desc, ttipm_problem** out) {
  return guarded([&]() -> int {
    if (!desc || !out) throw Error(TT_ERR_ARG, "NULL argument");
    Ctx& c = ctx_for(nullptr);
    c.prec = GemmPrec::F64;
    auto p = std::make_unique<ttipm_problem>();
    if (desc->kind == TTIPM_GENERIC) {
      auto get = [&](const tt_view& v, const char* name, std::unique_ptr<TT>& hold) -> const TT* {
        check_view(&v, name);
        hold = std::make_unique<TT>(tt_from_view(v, c));
        return hold.get();
      };
      std::unique_ptr<TT> h[9];
      GenericSdp g;
      g.C = get(desc->C, "C", h[0]);
      g.Aeq = get(desc->Aeq, "Aeq", h[1]);
      g.AeqT = get(desc->AeqT, "AeqT", h[2]);
      g.Beq = get(desc->Beq, "Beq", h[3]);
      g.KY = get(desc->KY, "KY", h[4]);
      if (desc->Aineq.d > 0) {
        g.Aineq = get(desc->Aineq, "Aineq", h[5]);
        g.AineqT = get(desc->AineqT, "AineqT", h[6]);
        g.Bineq = get(desc->Bineq, "Bineq", h[7]);
        g.KT = get(desc->KT, "KT", h[8]);
        g.sense = desc->ineq_sense;
        g.q = desc->q;
        g.x0_ineq = desc->x0_ineq;
        g.t0_ineq = desc->t0_ineq;
      }
      if (!(desc->lam0 > 0.0)) throw Error(TT_ERR_ARG, "lam0 must be positive");
      g.lam0 = desc->lam0;
      p->P = build_problem_generic(g, c);
    } else {
      check_view(&desc->graph, "graph");
      if (desc->graph.m_out != 2 || desc->graph.m_in != 2) throw Error(TT_ERR_ARG, "graph must have 2 x 2 modes");
      TT G = tt_from_view(desc->graph, c);
      std::unique_ptr<TT> nd;
      if (desc->kind == TTIPM_CC) {
        check_view(&desc->negdeg, "negdeg");
        nd = std::make_unique<TT>(tt_from_view(desc->negdeg, c));
      }
      p->P = build_problem(desc->kind, G, nd.get(), c);
    }
    c.sync();
    *out = p.release();
    return TT_OK;
  });
}

void ttipm_problem_destroy(ttipm_problem* p) { delete p; }

int ttipm_state_create(const ttipm_problem* p, const ttipm_params* prm, ttipm_state** out) {
  return guarded([&]() -> int {
    if (!p || !prm || !out) throw Error(TT_ERR_ARG, "NULL argument");
    Ctx& c = ctx_for(nullptr);
    auto s = std::make_unique<ttipm_state>();
    init_state(p->P, *prm, s->S, c);
    s->d = p->P.d;
    c.sync();
    *out = s.release();
    return TT_OK;
  });
}

void ttipm_state_destroy(ttipm_state* s) { delete s; }

int ttipm_step(ttipm_problem* p, ttipm_state* s, const ttipm_params* prm, ttipm_step_info* info, void* stream) {
  return guarded([&]() -> int {
    if (!p || !s || !prm) throw Error(TT_ERR_ARG, "NULL argument");
    Ctx& c = ctx_for(stream);
    c.prec = GemmPrec::F64;
    ttipm_step_info inf{};
    ipm_step(p->P, s->S, *prm, inf, c);
    if (info) *info = inf;
    if (!std::isfinite(inf.pobj) || !std::isfinite(inf.dobj)) throw Error(TT_ERR_NUMERIC, "non-finite objective");
    return TT_OK;
  });
}

int ttipm_solve(ttipm_problem* p, ttipm_state* s, const ttipm_params* prm, ttipm_result* res, ttipm_step_info* log,
                int32_t log_cap, void* stream) {
  return guarded([&]() -> int {
    if (!p || !s || !prm || !res) throw Error(TT_ERR_ARG, "NULL argument");
    Ctx& c = ctx_for(stream);
    c.prec = GemmPrec::F64;
    const auto t0 = std::chrono::steady_clock::now();
    auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    ttipm_result r{};
    r.time_to_gap = -1.0;
    r.status = TT_ERR_NOT_CONVERGED;
    int it = 0;
    int short_steps = 0;
    for (;; ++it) {
      ttipm_step_info m{};
      ipm_measures(p->P, s->S, m, c);
      const bool at_mark = m.rel_gap <= prm->eps_gap && m.eps_p <= 2 * prm->eps_gap && m.eps_d <= 2 * prm->eps_gap;
      if (at_mark && r.time_to_gap < 0) r.time_to_gap = elapsed();
      r.pobj = m.pobj;
      r.dobj = m.dobj;
      r.rel_gap = m.rel_gap;
      r.eps_p = m.eps_p;
      r.eps_d = m.eps_d;
      r.norm_rp = m.norm_rp;
      r.norm_rd = m.norm_rd;
      r.xz = m.xz;
      r.absolute_met = ipm_absolute_done(m, *prm) ? 1 : 0;
      // relative criteria; with the finishing phase on, the solve goes on
      // from there to the absolute ones and any later stop returns the last
      // accepted iterate, which still meets the relative criteria
      const bool rel_done = ipm_relative_done(m, *prm);
      if (rel_done) r.status = TT_OK;
      if (rel_done && (!prm->finish || ipm_absolute_done(m, *prm))) break;
      if (it >= prm->max_iter) break;
      // Stall: the TT direction no longer admits a step (both step lengths
      // below 1e-3 in five consecutive iterations: from the scaled identity
      // start, the first steps on large instances can be of order 1/n before
      // the iteration recovers), or an iterate lost positive definiteness in
      // the step-length test; the last accepted iterate is the result.
      if (short_steps >= 5) {
        if (!rel_done) r.status = TT_ERR_NOT_CONVERGED;
        break;
      }
      ttipm_step_info inf{};
      try {
        ipm_step(p->P, s->S, *prm, inf, c, &m);
      } catch (const Error& e) {
        if (e.code != TT_ERR_NOT_PD) throw;
        r.status = TT_ERR_NOT_PD;
        if (prm->verbose) std::fprintf(stderr, "stop: %s\n", e.what());
        break;
      }
      short_steps = (inf.alpha_p < 1e-3 && inf.alpha_d < 1e-3) ? short_steps + 1 : 0;
      r.finish_iterations += inf.finishing;
      if (log && it < log_cap) log[it] = inf;
      if (prm->verbose)
        std::fprintf(stderr,
                     "it %2d %s mu %.2e pobj %+.10e dobj %+.10e gap %.2e ep %.1e ed %.1e ap %.3e/%.3e ad %.3e/%.3e "
                     "bt %d g4 %d fin %d nu %.0e psi %.2e zx %.1e/%.1e zz %.1e/%.1e nres %.1e rf %d rX %d rY %d rZ %d rW %d sw %d/%d "
                     "kr %d sig %.2e eta %.1e t %.3fs\n",
                     inf.iter, inf.direction ? "aho" : (inf.xz_fallback ? "xz*" : "xz "), inf.mu, inf.pobj, inf.dobj, inf.rel_gap, inf.eps_p,
                     inf.eps_d, inf.alpha_p, inf.alpha_p_max, inf.alpha_d, inf.alpha_d_max, inf.backtracks,
                     inf.g4_retries, inf.finishing + inf.finish_rejected, inf.nu, inf.psi, inf.zeta_x, inf.zeta_x_cap, inf.zeta_z, inf.zeta_z_cap, inf.newton_res,
                     inf.refine_sweeps, inf.rank_x, inf.rank_y, inf.rank_z, inf.rank_w, inf.sweeps_pred, inf.sweeps_corr,
                     inf.krylov_iters, inf.sigma, inf.eta, inf.t_total);
      if (!std::isfinite(inf.pobj)) throw Error(TT_ERR_NUMERIC, "non-finite objective");
    }
    r.iterations = it;
    r.time_total = elapsed();
    *res = r;
    return TT_OK;
  });
}

int ttipm_state_export(const ttipm_state* s, int32_t which, int32_t* ranks_out, double* host_out, size_t cap,
                       size_t* needed) {
  return guarded([&]() -> int {
    if (!s || !ranks_out) throw Error(TT_ERR_ARG, "NULL argument");
    const TT* t = nullptr;
    switch (which) {
      case 'X': t = &s->S.X; break;
      case 'Y': t = &s->S.Y; break;
      case 'Z': t = &s->S.Z; break;
      case 'T': t = &s->S.T; break;
      case 'x': t = &s->S.dX; break;
      case 'y': t = &s->S.dY; break;
      case 'z': t = &s->S.dZ; break;
      case 't': t = &s->S.dT; break;
      default: throw Error(TT_ERR_ARG, "which must be one of X Y Z T x y z t");
    }
    if (t->d == 0) throw Error(TT_ERR_ARG, "iterate not present");
    size_t total = 0;
    for (int k = 0; k < t->d; ++k) total += (size_t)t->core_size(k);
    if (needed) *needed = total;
    for (int k = 0; k <= t->d; ++k) ranks_out[k] = t->r[k];
    if (!host_out || cap < total) return (int)TT_ERR_ARG;
    Ctx& c = ctx_for(nullptr);
    size_t off = 0;
    for (int k = 0; k < t->d; ++k) {
      TT_HIP(hipMemcpyAsync(host_out + off, t->core(k), sizeof(double) * t->core_size(k), hipMemcpyDeviceToHost, c.s));
      off += (size_t)t->core_size(k);
    }
    c.sync();
    return TT_OK;
  });
}

int ttipm_state_import(ttipm_state* s, int32_t which, const int32_t* ranks, const double* host_in, size_t count) {
  return guarded([&]() -> int {
    if (!s || !ranks || !host_in) throw Error(TT_ERR_ARG, "NULL argument");
    TT* t = nullptr;
    switch (which) {
      case 'X': t = &s->S.X; break;
      case 'Y': t = &s->S.Y; break;
      case 'Z': t = &s->S.Z; break;
      case 'T': t = &s->S.T; break;
      default: throw Error(TT_ERR_ARG, "which must be one of X Y Z T");
    }
    if (t->d == 0) throw Error(TT_ERR_ARG, "iterate not present in this state");
    const int d = t->d;
    if (ranks[0] != 1 || ranks[d] != 1) throw Error(TT_ERR_ARG, "boundary ranks must be 1");
    size_t total = 0;
    for (int k = 0; k < d; ++k) {
      if (ranks[k + 1] < 1) throw Error(TT_ERR_ARG, "ranks must be positive");
      total += (size_t)ranks[k] * t->mo * t->mi * ranks[k + 1];
    }
    if (count != total) throw Error(TT_ERR_ARG, "core data size does not match the ranks");
    std::vector<std::vector<double>> cores(d);
    size_t off = 0;
    for (int k = 0; k < d; ++k) {
      const size_t n = (size_t)ranks[k] * t->mo * t->mi * ranks[k + 1];
      cores[k].assign(host_in + off, host_in + off + n);
      off += n;
    }
    Ctx& c = ctx_for(nullptr);
    *t = tt_from_host(cores, std::vector<int>(ranks, ranks + d + 1), t->mo, t->mi, c);
    c.sync();
    return TT_OK;
  });
}

int tt_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, int32_t seed, tt_mlp** out) {
  return guarded([&]() -> int {
    if (!out) throw Error(TT_ERR_ARG, "out is NULL");
    if (in_dim < 1 || hidden < 1 || out_dim < 1) throw Error(TT_ERR_ARG, "network dimensions");
    auto m = std::make_unique<tt_mlp>();
    Ctx& c = ctx_for(nullptr);
    m->net.init(in_dim, hidden, out_dim, (unsigned long long)(unsigned)seed, c);
    *out = m.release();
    return TT_OK;
  });
}

void tt_mlp_destroy(tt_mlp* m) { delete m; }

int64_t tt_mlp_num_params(const tt_mlp* m) { return m ? (int64_t)m->net.nparams : 0; }

int tt_mlp_get_params(const tt_mlp* m, float* host, int64_t count) {
  return guarded([&]() -> int {
    if (!m || !host || count != m->net.nparams) throw Error(TT_ERR_ARG, "parameter buffer");
    Ctx& c = ctx_for(nullptr);
    TT_HIP(hipMemcpyAsync(host, m->net.params.get(), sizeof(float) * count, hipMemcpyDeviceToHost, c.s));
    c.sync();
    return TT_OK;
  });
}

int tt_mlp_set_params(tt_mlp* m, const float* host, int64_t count) {
  return guarded([&]() -> int {
    if (!m || !host || count != m->net.nparams) throw Error(TT_ERR_ARG, "parameter buffer");
    Ctx& c = ctx_for(nullptr);
    TT_HIP(hipMemcpyAsync(m->net.params.get(), host, sizeof(float) * count, hipMemcpyHostToDevice, c.s));
    c.sync();
    return TT_OK;
  });
}

static MlpBatch as_batch(const tt_mlp_batch* b, const tt_mlp* m) {
  MlpBatch mb;
  if (b) {
    if (b->N < 1 || b->P < 1 || b->n < 1 || !b->F || !b->R || !b->Y || !b->S || !b->W)
      throw Error(TT_ERR_ARG, "invalid tt_mlp_batch");
    mb = MlpBatch{b->N, b->P, b->n, b->F, b->R, b->Y, b->S, b->W};
  } else {
    const Mlp& net = m->net;
    if (net.ds_N < 1) throw Error(TT_ERR_ARG, "the collected dataset is empty");
    mb = MlpBatch{(int)net.ds_N, net.ds_P, net.ds_n, net.dsF.get(), net.dsR.get(), net.dsY.get(), net.dsS.get(),
                  net.dsW.get()};
  }
  if (mb.n * mb.n != m->net.out || mb.n * mb.n + 5 != m->net.in)
    throw Error(TT_ERR_ARG, "batch block size does not match the network (in = n*n + 5, out = n*n)");
  return mb;
}

int tt_mlp_loss_grad(tt_mlp* m, const tt_mlp_batch* b, double* loss, float* grad_host, void* stream) {
  return guarded([&]() -> int {
    if (!m) throw Error(TT_ERR_ARG, "mlp is NULL");
    Ctx& c = ctx_for(stream);
    const MlpBatch mb = as_batch(b, m);
    const double l = m->net.loss_grad(mb, c);
    if (loss) *loss = l;
    if (grad_host) {
      TT_HIP(hipMemcpyAsync(grad_host, m->net.grad.get(), sizeof(float) * m->net.nparams, hipMemcpyDeviceToHost, c.s));
      c.sync();
    }
    return TT_OK;
  });
}

int tt_mlp_collect(tt_mlp* m, const tt_local_op* K, const float* context, int32_t nprobe, int32_t seed, int64_t cap,
                   void* stream) {
  return guarded([&]() -> int {
    if (!m) throw Error(TT_ERR_ARG, "mlp is NULL");
    check_local_op(K);
    if (nprobe < 1) throw Error(TT_ERR_ARG, "nprobe must be >= 1");
    Ctx& c = ctx_for(stream);
    c.prec = GemmPrec::F64;
    const int n = K->L * K->m;
    if (n * n != m->net.out || n * n + 5 != m->net.in) throw Error(TT_ERR_ARG, "block size does not match the network");
    BlockJacobi raw, inv;
    raw.init(K->r, K->rp, K->m, K->L, c);
    for (int b = 0; b < K->nblocks; ++b) {
      const tt_local_block& B = K->blocks[b];
      BlockJacobi::Op ch[2];
      for (int q = 0; q < B.nchain; ++q) ch[q] = {B.op[q].phiL, B.op[q].core, B.op[q].phiR, B.op[q].R, B.op[q].Rp};
      raw.add(B.row, B.col, B.coeff, ch, B.nchain, c);
    }
    inv.copy_from(raw, c);
    inv.invert(c);
    float ctx[4] = {0.f, 0.f, 0.f, 0.f};
    if (context) for (int q = 0; q < 4; ++q) ctx[q] = context[q];
    FBuf F, R, Y, S, W;
    mlp_block_data(raw, inv, [&](const double* xv, double* yv) { generic_matvec(K, xv, yv, c); }, ctx, nprobe,
                   (unsigned long long)(unsigned)seed, F, R, Y, S, W, c);
    const MlpBatch mb{K->r * K->rp, nprobe, n, F.get(), R.get(), Y.get(), S.get(), W.get()};
    m->net.append(mb, cap, c);
    return TT_OK;
  });
}

int tt_mlp_dataset_size(const tt_mlp* m, int64_t* n_blocks) {
  return guarded([&]() -> int {
    if (!m || !n_blocks) throw Error(TT_ERR_ARG, "NULL argument");
    *n_blocks = m->net.ds_N;
    return TT_OK;
  });
}

int tt_mlp_train(tt_mlp* m, const tt_mlp_batch* data, int32_t epochs, int32_t batch, float lr, int32_t seed,
                 double* loss_hist, void* stream) {
  return guarded([&]() -> int {
    if (!m) throw Error(TT_ERR_ARG, "mlp is NULL");
    if (epochs < 0 || batch < 1 || !(lr > 0.f)) throw Error(TT_ERR_ARG, "training parameters");
    Ctx& c = ctx_for(stream);
    const MlpBatch mb = as_batch(data, m);
    std::vector<double> hist;
    mlp_train(m->net, mb, epochs, batch, lr, (unsigned long long)(unsigned)seed, hist, c);
    if (loss_hist) for (int e = 0; e < epochs; ++e) loss_hist[e] = hist[e];
    return TT_OK;
  });
}

int tt_mlp_eval(tt_mlp* m, const tt_mlp_batch* data, double* loss, void* stream) {
  return guarded([&]() -> int {
    if (!m || !loss) throw Error(TT_ERR_ARG, "NULL argument");
    Ctx& c = ctx_for(stream);
    *loss = m->net.loss_grad(as_batch(data, m), c);
    return TT_OK;
  });
}

}  // extern "C"
