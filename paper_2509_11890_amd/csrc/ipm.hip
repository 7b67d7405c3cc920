// TT interior-point method driver (see ipm.hpp).  The loop and all decisions
// (ranks, step lengths, stopping) are host logic; every arithmetic operation on
// TT data runs in the library's kernels.
#include "ipm.hpp"
#include "mlp.hpp"

#include <algorithm>
#include <deque>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <random>

#include "blocked.hpp"
#include "dense.hpp"
#include "ttops.hpp"

namespace ttipm {

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

const std::vector<double> I4 = {1, 0, 0, 1};
const std::vector<double> J4 = {1, 1, 1, 1};
const std::vector<double> E4 = {1, 0, 0, 0};

std::vector<double> outer4(const std::vector<double>& u, const std::vector<double>& v) {
  std::vector<double> o(16);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) o[i * 4 + j] = u[i] * v[j];
  return o;
}

// Compress an exactly built TT (sums of elementary terms) to minimal ranks.
void compress(TT& t, Ctx& c) {
  double nrm = tt_norm(t, c);
  if (nrm > 0) tt_round_abs(t, 1e-14 * nrm, 1 << 30, c);
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

// Rounding with the spectral shift of Cor. 1: round at tol / (1 + ||S||_F) and
// add zeta S; keep the unrounded tensor if the rank does not drop (and is
// within the cap).  Cor. 1 budgets the error the tolerance allows
// (zeta <= tol / (1 + ||S||_F)); a binding rank cap discards more.  The
// eigenvalue bound of Cor. 1 (Weyl) holds for any zeta, so with shift_all the
// whole zeta is added and positive definiteness is kept; its cap-forced part
// then moves every affine residual by up to zeta_cap ||A S|| (for MaxCut every
// diagonal entry of X), which the windowed residual control of the update
// watches.  Without shift_all only the tolerance part is added.
struct ShiftInfo {
  double zeta = 0.0;      // ||M - M~||_F of the rounding (0 if the tensor was kept)
  double zeta_tol = 0.0;  // the part within the tolerance budget
};

TT round_shift(TT v, double tol, const TT* shift, int cap, Ctx& c, ShiftInfo* si, bool shift_all = true) {
  const double nS = shift ? tt_norm(*shift, c) : 0.0;
  const int r0 = v.max_rank();
  TT vt = tt_clone(v, c);
  double zeta_tol = 0.0;
  const double zeta = tt_round_abs(vt, tol / (1.0 + nS), cap, c, nullptr, &zeta_tol);
  if (vt.max_rank() >= r0 && r0 <= cap) {
    if (si) *si = ShiftInfo{};
    return v;
  }
  if (si) {
    si->zeta = zeta;
    si->zeta_tol = zeta_tol;
  }
  const double z = shift_all ? zeta : zeta_tol;
  if (shift && z > 0) return tt_add({&vt, shift}, {1.0, z}, c);
  return vt;
}

}  // namespace

// ---------------------------------------------------------------------------
// problem encodings (Sec. 4)
// ---------------------------------------------------------------------------
// Non-idle multiplier masks P_Y = I - K_Y, P_T = I - K_T and whether they are
// disjoint (P_Y P_T = 0, checked on the diagonal P_Y P_T vec_TT(J) of the two
// diagonal masks): the condition of the combined multiplier storage of Sec. 3.5.
void multiplier_masks(Problem& P, Ctx& c) {
  P.PY = tt_add({&P.I16, &P.KY}, {1.0, -1.0}, c);
  P.PT = tt_add({&P.I16, &P.KT}, {1.0, -1.0}, c);
  compress(P.PY, c);
  compress(P.PT, c);
  TT Jvec = tt_rank1(P.d, 4, 1, J4, c);
  TT t = tt_matvec(P.PT, Jvec, c);
  TT b = tt_matvec(P.PY, t, c);
  P.masks_disjoint = tt_norm(b, c) <= 1e-12 * tt_norm(Jvec, c);
}

Problem build_problem(int kind, const TT& G, const TT* negdeg, Ctx& c) {
  TT_REQUIRE(G.mo == 2 && G.mi == 2, "graph must be a TT matrix with 2 x 2 modes");
  Problem P;
  P.kind = kind;
  P.d = G.d;
  const int d = G.d;
  P.n = std::ldexp(1.0, d);
  P.Ivec = tt_rank1(d, 4, 1, I4, c);
  P.I2 = tt_rank1(d, 2, 2, {1, 0, 0, 1}, c);
  {
    std::vector<double> i16(16, 0.0);
    for (int i = 0; i < 4; ++i) i16[i * 4 + i] = 1.0;
    P.I16 = tt_rank1(d, 4, 4, i16, c);
  }
  TT Jvec = tt_rank1(d, 4, 1, J4, c);
  TT Evec = tt_rank1(d, 4, 1, E4, c);
  TT JmI = tt_add({&Jvec, &P.Ivec}, {1.0, -1.0}, c);
  if (kind == TTIPM_MAXCUT) {
    // C = (diag_TT(A_G 1) - A_G) / 4, A_eq = diag_TT(vec_TT I), B_eq = vec_TT I, K_Y = diag_TT(vec_TT(J - I))
    TT ones2 = tt_rank1(d, 2, 1, {1, 1}, c);
    TT deg = tt_matvec(G, ones2, c);
    TT D = tt_diag(deg, c);
    TT Cm = tt_add({&D, &G}, {0.25, -0.25}, c);
    P.C = tt_as_vector(Cm, c);
    P.Aeq = tt_diag(P.Ivec, c);
    P.AeqT = tt_clone(P.Aeq, c);
    P.Beq = tt_clone(P.Ivec, c);
    P.KY = tt_diag(JmI, c);
    P.lam0 = 1.0;
  } else if (kind == TTIPM_THETA) {
    // C = J, A_eq = diag_TT(vec_TT A_G) + vec_TT(E_11) vec_TT(I)^T, B_eq = vec_TT(E_11),
    // K_Y = diag_TT(vec_TT(J - A_G) - B_eq)
    TT Avec = tt_as_vector(G, c);
    TT part1 = tt_diag(Avec, c);
    TT p2 = tt_rank1(d, 4, 4, outer4(E4, I4), c);
    TT p2t = tt_rank1(d, 4, 4, outer4(I4, E4), c);
    P.Aeq = tt_add({&part1, &p2}, {1.0, 1.0}, c);
    P.AeqT = tt_add({&part1, &p2t}, {1.0, 1.0}, c);
    P.Beq = tt_clone(Evec, c);
    TT mask = tt_add({&Jvec, &Avec, &Evec}, {1.0, -1.0, -1.0}, c);
    P.KY = tt_diag(mask, c);
    P.C = tt_clone(Jvec, c);
    P.lam0 = 2.0;
  } else if (kind == TTIPM_CC) {
    // C = W + diag_TT(C^- 1); A_eq = diag_TT(vec_TT I), K_Y = diag_TT(vec_TT(J - I));
    // A_ineq = diag_TT(vec_TT(J - I)) with the >= convention, K_T = diag_TT(vec_TT I)
    TT_REQUIRE(negdeg != nullptr && negdeg->mo == 2 && negdeg->mi == 1, "negdeg TT vector with mode 2");
    TT Dm = tt_diag(*negdeg, c);
    TT Cm = tt_add({&G, &Dm}, {1.0, 1.0}, c);
    P.C = tt_as_vector(Cm, c);
    P.Aeq = tt_diag(P.Ivec, c);
    P.AeqT = tt_clone(P.Aeq, c);
    P.Beq = tt_clone(P.Ivec, c);
    P.KY = tt_diag(JmI, c);
    P.ineq = true;
    P.sense = -1.0;
    P.Aineq = tt_diag(JmI, c);
    P.AineqT = tt_clone(P.Aineq, c);
    P.KT = tt_diag(P.Ivec, c);
    P.Bineq = tt_clone(P.Ivec, c);
    tt_scale(P.Bineq, 0.0, c);
    P.oneT = tt_clone(JmI, c);
    P.q = P.n * P.n - P.n;
    P.lam0 = 2.0;
    P.x0_ineq = P.lam0 / 10.0;
  } else {
    throw Error(TT_ERR_ARG, "unknown problem kind");
  }
  compress(P.C, c);
  compress(P.Aeq, c);
  compress(P.AeqT, c);
  compress(P.KY, c);
  if (P.ineq) {
    compress(P.Aineq, c);
    compress(P.AineqT, c);
    compress(P.KT, c);
    compress(P.oneT, c);
    multiplier_masks(P, c);
  }
  P.normB = tt_norm(P.Beq, c);
  P.normC = tt_norm(P.C, c);
  return P;
}

Problem build_problem_generic(const GenericSdp& g, Ctx& c) {
  auto vec = [](const TT* t, const char* name) {
    TT_REQUIRE(t && t->mo == 4 && t->mi == 1, std::string(name) + " must be a vec_TT vector (mode 4)");
  };
  auto op = [](const TT* t, const char* name) {
    TT_REQUIRE(t && t->mo == 4 && t->mi == 4, std::string(name) + " must be an operator on vec_TT (4 x 4 modes)");
  };
  vec(g.C, "C");
  vec(g.Beq, "B_eq");
  op(g.Aeq, "A_eq");
  op(g.AeqT, "A_eq^T");
  op(g.KY, "K_Y");
  const int d = g.C->d;
  for (const TT* t : {g.Aeq, g.AeqT, g.Beq, g.KY})
    TT_REQUIRE(t->d == d, "every TT of the problem must have the same number of cores");
  Problem P;
  P.kind = TTIPM_GENERIC;
  P.d = d;
  P.n = std::ldexp(1.0, d);
  P.Ivec = tt_rank1(d, 4, 1, I4, c);
  P.I2 = tt_rank1(d, 2, 2, {1, 0, 0, 1}, c);
  {
    std::vector<double> i16(16, 0.0);
    for (int i = 0; i < 4; ++i) i16[i * 4 + i] = 1.0;
    P.I16 = tt_rank1(d, 4, 4, i16, c);
  }
  P.C = tt_clone(*g.C, c);
  P.Aeq = tt_clone(*g.Aeq, c);
  P.AeqT = tt_clone(*g.AeqT, c);
  P.Beq = tt_clone(*g.Beq, c);
  P.KY = tt_clone(*g.KY, c);
  P.lam0 = g.lam0;
  if (g.Aineq) {
    op(g.Aineq, "A_ineq");
    op(g.AineqT, "A_ineq^T");
    op(g.KT, "K_T");
    vec(g.Bineq, "B_ineq");
    for (const TT* t : {g.Aineq, g.AineqT, g.KT, g.Bineq})
      TT_REQUIRE(t->d == d, "every TT of the problem must have the same number of cores");
    TT_REQUIRE(g.sense == 1.0 || g.sense == -1.0, "ineq_sense must be +1 or -1");
    P.ineq = true;
    P.sense = g.sense;
    P.Aineq = tt_clone(*g.Aineq, c);
    P.AineqT = tt_clone(*g.AineqT, c);
    P.KT = tt_clone(*g.KT, c);
    P.Bineq = tt_clone(*g.Bineq, c);
    // active inequality mask 1_T = vec_TT(J) - K_T vec_TT(J)
    TT Jvec = tt_rank1(d, 4, 1, J4, c);
    TT KJ = tt_matvec(P.KT, Jvec, c);
    P.oneT = tt_add({&Jvec, &KJ}, {1.0, -1.0}, c);
    P.q = g.q;
    P.x0_ineq = g.x0_ineq;
    P.t0_ineq = g.t0_ineq;
  }
  compress(P.C, c);
  compress(P.Aeq, c);
  compress(P.AeqT, c);
  compress(P.KY, c);
  if (P.ineq) {
    compress(P.Aineq, c);
    compress(P.AineqT, c);
    compress(P.KT, c);
    compress(P.oneT, c);
    multiplier_masks(P, c);
  }
  P.normB = tt_norm(P.Beq, c);
  P.normC = tt_norm(P.C, c);
  return P;
}

void init_state(const Problem& P, const ttipm_params& prm, State& S, Ctx& c) {
  // Sec. 5.1: X = Z = lambda* I, Y = 0; with inequalities X = lambda* I + (alpha_p/10) A_ineq(J),
  // T = lambda*_ineq A_ineq(J) (reading: alpha_p = lambda* for A_G = J - I).
  S.seed = (unsigned long long)(unsigned)prm.seed;
  S.X = tt_clone(P.Ivec, c);
  tt_scale(S.X, P.lam0, c);
  S.Z = tt_clone(P.Ivec, c);
  tt_scale(S.Z, P.lam0, c);
  S.Y = tt_clone(P.Ivec, c);
  tt_scale(S.Y, 0.0, c);
  if (P.ineq) {
    TT Jvec = tt_rank1(P.d, 4, 1, J4, c);
    TT AJ = tt_matvec(P.Aineq, Jvec, c);
    compress(AJ, c);
    TT X2 = tt_add({&S.X, &AJ}, {1.0, P.x0_ineq}, c);
    S.X = std::move(X2);
    S.T = tt_clone(AJ, c);
    tt_scale(S.T, P.t0_ineq, c);
  }
  S.eta = prm.eta0;
  S.iter = 0;
  S.has_W = false;
  S.has_EX = S.has_EZ = false;
}

// ---------------------------------------------------------------------------
// step length (Sec. 3.4): extreme generalised Rayleigh quotient in TT form,
// solved by a two-site DMRG sweep.  At each pair of cores the projected pencil
// (dM^, M^) is reduced with the Cholesky factor of M^ and its smallest
// eigenpair is taken by Lanczos, warm-started from the current E projected on
// the pair's frame; the pair is then split by a truncated SVD, which adapts the
// rank of E up to `rank`.
// ---------------------------------------------------------------------------
namespace {

// merged two-site operator core [R_k][(i,i')][(j,j')][R_{k+2}] of a TT matrix with 2 x 2 modes
void merge_pair(const TT& M, int k, DevBuf& out, Ctx& c) {
  const int R0 = M.r[k], R1 = M.r[k + 1], R2 = M.r[k + 2];
  DevBuf tmp((size_t)R0 * 4 * 4 * R2);
  gemm(gemm_nn(R0 * 4, 4 * R2, R1, M.core(k), R1, M.core(k + 1), 4 * R2, tmp.get(), 4 * R2), c.s, &c.ws,
       GemmPrec::F64);
  out.reserve((size_t)R0 * 16 * R2);
  // [a][i][j][i'][j'][g] -> [a][i][i'][j][j'][g]
  permute(tmp.get(), out.get(), {R0, 2, 2, 2, 2, R2}, {0, 1, 3, 2, 4, 5}, c.s);
}

// y = L^T x for a lower triangular row-major L (only the lower triangle is read)
__global__ void trmv_lt_kernel(const double* L, int p, const double* x, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p) return;
  double acc = 0.0;
  for (int j = i; j < p; ++j) acc += L[(long)j * p + i] * x[j];
  y[i] = acc;
}

__global__ void scale_rows_kernel(double* A, int rows, int cols, long ld, const double* s) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)rows * cols) return;
  const int i = (int)(t / cols), j = (int)(t % cols);
  A[i * ld + j] *= s[i];
}

__global__ void scale_cols_kernel(double* A, int rows, int cols, long ld, const double* s) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)rows * cols) return;
  const int i = (int)(t / cols), j = (int)(t % cols);
  A[i * ld + j] *= s[j];
}

// smallest eigenpair of the pencil (D, M) (p x p, row-major, symmetrised in place):
// returns lambda and writes the M-normalised direction into e (p).  e0 (or
// nullptr): an approximate eigenvector that starts the Lanczos iteration.
// pencils from this size on use the blocked (GEMM-based) factorisations
constexpr int kPencilBlocked = 96;

double pencil_min(double* Mm, double* D, int p, double* e, Ctx& c, const double* e0 = nullptr) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblocks((long)p * p, 256)), dim3(256), 0, c.s, Mm, p);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblocks((long)p * p, 256)), dim3(256), 0, c.s, D, p);
  TT_HIP(hipGetLastError());
  // Pencils of a few hundred unknowns use the GEMM-based blocked Cholesky and
  // triangular solves; the single-workgroup kernels win only for small ones.
  const bool blocked = p >= kPencilBlocked || !dense_small_fits_lds(p);
  BlockedFactors f;
  int* st = nullptr;
  if (blocked) {
    if (chol_blocked(Mm, p, f, c) != 0)
      throw Error(TT_ERR_NOT_PD, "projected iterate is not positive definite (step length)");
  } else {
    // the status is read back with the eigenvalue at the end: a failed
    // factorisation only wastes the work queued after it
    c.ired.reserve((size_t)p + 8);
    st = reinterpret_cast<int*>(c.ired.get());
    dense_cholesky(Mm, p, st, c.s);
  }
  auto solve_L = [&](double* B, int nrhs, bool trans) {
    if (blocked)
      trsm_blocked(Mm, p, f, B, nrhs, trans, c);
    else
      dense_trsm_lower(Mm, p, B, nrhs, trans, c.s);
  };
  DevBuf Bt((size_t)p * p), work((size_t)p * (std::min(p, 128) + 1)), lam(1);
  solve_L(D, p, false);                                      // L^{-1} D
  permute(D, Bt.get(), {p, p}, {1, 0}, c.s);                 // (L^{-1} D)^T = D L^{-T}
  solve_L(Bt.get(), p, false);                               // L^{-1} D L^{-T}
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblocks((long)p * p, 256)), dim3(256), 0, c.s, Bt.get(), p);
  TT_HIP(hipGetLastError());
  // smallest eigenpair of the reduced pencil (Lanczos, started from v = L^T e0
  // when given), then e = L^{-T} v
  if (e0) {
    hipLaunchKernelGGL(trmv_lt_kernel, dim3(nblocks(p, 256)), dim3(256), 0, c.s, Mm, p, e0, e);
    TT_HIP(hipGetLastError());
  }
  dense_sym_min_eig(Bt.get(), p, e, lam.get(), work.get(), c.s, 128, 8, 1e-12, e0 != nullptr);
  solve_L(e, 1, true);
  double lmin = 0.0;
  int hst = 0;
  TT_HIP(hipMemcpyAsync(&lmin, lam.get(), sizeof(double), hipMemcpyDeviceToHost, c.s));
  if (st) TT_HIP(hipMemcpyAsync(&hst, st, sizeof(int), hipMemcpyDeviceToHost, c.s));
  c.sync();
  if (hst != 0) throw Error(TT_ERR_NOT_PD, "projected iterate is not positive definite (step length)");
  return lmin;
}

}  // namespace

double min_gen_eig(const TT& Mv, const TT& dMv, BlockTT& E, bool& have_E, int rank, int sweeps, int kick,
                   unsigned long long seed, Ctx& c) {
  const int d = Mv.d;
  TT M = tt_as_matrix(Mv, 2, c);
  TT dM = tt_as_matrix(dMv, 2, c);
  if (!have_E) {
    // seeded random start of TT rank min(rank, 2), right-orthogonalised; DMRG grows the rank
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<int> rk(d + 1, 1);
    for (int k = 1; k < d; ++k) rk[k] = std::min(2, rank);
    std::vector<std::vector<double>> cores(d);
    for (int k = 0; k < d; ++k) {
      cores[k].resize((size_t)rk[k] * 2 * rk[k + 1]);
      for (double& x : cores[k]) x = nd(rng);
    }
    TT e0 = tt_from_host(cores, rk, 2, 1, c);
    E = block_from_frame(e0, 1, c);
    have_E = true;
  }
  if (d == 1) {
    // a single core: the local problem is the whole pencil
    DevBuf Ml(4), Dl(4), e(2);
    TT_HIP(hipMemcpyAsync(Ml.get(), M.core(0), 4 * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    TT_HIP(hipMemcpyAsync(Dl.get(), dM.core(0), 4 * sizeof(double), hipMemcpyDeviceToDevice, c.s));
    return pencil_min(Ml.get(), Dl.get(), 2, e.get(), c);
  }
  if (!E.cores[0].get()) {
    // a fresh start has no weights in core 0 yet: the first pair starts Lanczos
    // from its fixed pseudo-random vector
    E.cores[0].reserve((size_t)2 * E.r[1]);
    fill((long)2 * E.r[1], 0.0, E.cores[0].get(), c.s);
  }
  std::vector<DevBuf> ML(d), MR(d), DL(d), DR(d);
  for (auto* v : {&ML, &DL}) { (*v)[0].reserve(1); fill(1, 1.0, (*v)[0].get(), c.s); }
  for (auto* v : {&MR, &DR}) { (*v)[d - 1].reserve(1); fill(1, 1.0, (*v)[d - 1].get(), c.s); }
  auto upd_right = [&](int k) {
    const int ra = E.r[k], ra2 = E.r[k + 1];
    MR[k - 1].reserve((size_t)ra * M.r[k] * ra);
    DR[k - 1].reserve((size_t)ra * dM.r[k] * ra);
    env_steps({{MR[k].get(), ra2, M.r[k + 1], ra2, E.cores[k].get(), 2, ra, M.core(k), M.r[k], 2, E.cores[k].get(),
                ra, MR[k - 1].get()},
               {DR[k].get(), ra2, dM.r[k + 1], ra2, E.cores[k].get(), 2, ra, dM.core(k), dM.r[k], 2,
                E.cores[k].get(), ra, DR[k - 1].get()}},
              false, c);
  };
  auto upd_left = [&](int k) {
    const int ra = E.r[k], ra2 = E.r[k + 1];
    ML[k + 1].reserve((size_t)ra2 * M.r[k + 1] * ra2);
    DL[k + 1].reserve((size_t)ra2 * dM.r[k + 1] * ra2);
    env_steps({{ML[k].get(), ra, M.r[k], ra, E.cores[k].get(), 2, ra2, M.core(k), M.r[k + 1], 2, E.cores[k].get(),
                ra2, ML[k + 1].get()},
               {DL[k].get(), ra, dM.r[k], ra, E.cores[k].get(), 2, ra2, dM.core(k), dM.r[k + 1], 2,
                E.cores[k].get(), ra2, DL[k + 1].get()}},
              true, c);
  };
  for (int k = d - 1; k > 0; --k) upd_right(k);
  double lam_best = 1e300;
  DevBuf M2, D2, Ml, Dl, e, e0, sg;
  // host copies of the singular values sent to the device, kept until the
  // synchronisation at the end (the pair steps do not wait for their copies)
  std::vector<std::vector<double>> sig_keep;
  // one sweep = left-to-right then right-to-left over the pairs (k, k+1);
  // further sweeps are skipped once the two passes of a sweep agree on the
  // smallest eigenvalue to 1e-9 (relative): the frame has converged
  for (int sw = 0; sw < sweeps; ++sw) {
    double lam_pass[2] = {1e300, 1e300};
    for (int pass = 0; pass < 2; ++pass) {
      const bool lr = (pass == 0);
      for (int step = 0; step < d - 1; ++step) {
        const int k = lr ? step : d - 2 - step;
        // block sits at k (lr) or k+1 (rl); frame: < k left-orth, > k+1 right-orth
        const int r = E.r[k], s = E.r[k + 2], p = r * 4 * s;
        merge_pair(M, k, M2, c);
        merge_pair(dM, k, D2, c);
        Ml.reserve((size_t)p * p);
        Dl.reserve((size_t)p * p);
        local_dense_ops({{ML[k].get(), r, M.r[k], M2.get(), 4, MR[k + 1].get(), s, M.r[k + 2], Ml.get()},
                         {DL[k].get(), r, dM.r[k], D2.get(), 4, DR[k + 1].get(), s, dM.r[k + 2], Dl.get()}},
                        c);
        e.reserve(p);
        // warm start: the current E on this pair's frame (the non-orthogonal
        // core carries the singular values of the last split)
        const int q0 = E.r[k + 1];
        e0.reserve(p);
        gemm(gemm_nn(2 * r, 2 * s, q0, E.cores[k].get(), q0, E.cores[k + 1].get(), 2 * s, e0.get(), 2 * s), c.s,
             &c.ws, GemmPrec::F64);
        const double lam = pencil_min(Ml.get(), Dl.get(), p, e.get(), c, e0.get());
        lam_best = std::min(lam_best, lam);
        lam_pass[pass] = std::min(lam_pass[pass], lam);
        // split the supercore [(r,i)][(i',s)] by a truncated SVD
        SvdOut sv;
        svd_rowmajor(e.get(), 2 * r, 2 * s, sv, c);
        double tot = 0;
        for (double x : sv.sigma) tot += x * x;
        int q = 1;
        for (int j = 1; j < sv.k; ++j)
          if (sv.sigma[j] > 1e-10 * std::sqrt(tot)) q = j + 1;
        q = std::max(1, std::min(q, rank));
        // Random kick ranks (Sec. 3.4): qk seeded random directions,
        // orthonormal to the kept ones, join the orthogonal core with zero
        // weight in its neighbour.  E is unchanged, but the next two-site
        // problem sees a larger frame, so a vector that has collapsed to a
        // low rank can still grow towards the true minimiser.
        const int qk = std::max(0, std::min(kick, (lr ? 2 * r : 2 * s) - q));
        const int rq = q + qk;
        const unsigned long long ks = seed * 1000003ull + (unsigned long long)((sw * 2 + pass) * 131 + k);
        E.cores[k].reserve((size_t)2 * r * rq);
        E.cores[k + 1].reserve((size_t)rq * 2 * s);
        sg.reserve(q);
        TT_HIP(hipMemcpyAsync(sg.get(), sv.sigma.data(), sizeof(double) * q, hipMemcpyHostToDevice, c.s));
        if (lr) {
          copy2d(sv.U.get(), sv.k, E.cores[k].get(), rq, 2 * r, q, c.s);                  // left-orthonormal
          TT_HIP(hipMemcpyAsync(E.cores[k + 1].get(), sv.Vt.get(), sizeof(double) * (size_t)q * 2 * s,
                                hipMemcpyDeviceToDevice, c.s));
          hipLaunchKernelGGL(scale_rows_kernel, dim3(nblocks((long)q * 2 * s, 256)), dim3(256), 0, c.s,
                             E.cores[k + 1].get(), q, 2 * s, (long)2 * s, sg.get());      // S Vt
          TT_HIP(hipGetLastError());
          if (qk > 0) {
            DevBuf G((size_t)qk * 2 * r), Gt((size_t)2 * r * qk);
            random_orth_rows(E.cores[k].get(), q, 1, rq, 2 * r, G.get(), qk, ks, c);
            permute(G.get(), Gt.get(), {qk, 2 * r}, {1, 0}, c.s);
            copy2d(Gt.get(), qk, E.cores[k].get() + q, rq, 2 * r, qk, c.s);
            fill((long)qk * 2 * s, 0.0, E.cores[k + 1].get() + (size_t)q * 2 * s, c.s);
          }
          E.r[k + 1] = rq;
          upd_left(k);
        } else {
          TT_HIP(hipMemcpyAsync(E.cores[k + 1].get(), sv.Vt.get(), sizeof(double) * (size_t)q * 2 * s,
                                hipMemcpyDeviceToDevice, c.s));                           // right-orthonormal
          copy2d(sv.U.get(), sv.k, E.cores[k].get(), rq, 2 * r, q, c.s);
          hipLaunchKernelGGL(scale_cols_kernel, dim3(nblocks((long)2 * r * q, 256)), dim3(256), 0, c.s,
                             E.cores[k].get(), 2 * r, q, (long)rq, sg.get());            // U S
          TT_HIP(hipGetLastError());
          if (qk > 0) {
            random_orth_rows(E.cores[k + 1].get(), q, 2 * s, 1, 2 * s, E.cores[k + 1].get() + (size_t)q * 2 * s, qk,
                             ks, c);
            DevBuf Z((size_t)2 * r * qk);
            fill((long)2 * r * qk, 0.0, Z.get(), c.s);
            copy2d(Z.get(), qk, E.cores[k].get() + q, rq, 2 * r, qk, c.s);
          }
          E.r[k + 1] = rq;
          upd_right(k + 1);
        }
        sig_keep.push_back(std::move(sv.sigma));   // device temporaries are recycled in stream order
      }
    }
    if (std::fabs(lam_pass[1] - lam_pass[0]) <= 1e-9 * std::max(std::fabs(lam_pass[0]), std::fabs(lam_pass[1])))
      break;
  }
  // leave E right-orthogonal with the block at 0 (core 0 is not orthogonal)
  E.pos = 0;
  E.blk.reserve((size_t)2 * E.r[1]);
  TT_HIP(hipMemcpyAsync(E.blk.get(), E.cores[0].get(), sizeof(double) * 2 * E.r[1], hipMemcpyDeviceToDevice, c.s));
  c.sync();
  return lam_best;
}

constexpr double kNoBound = 1e6;

namespace {

// Dense entries of a TT vector (row-major product of the cores; the first core
// is the most significant index).  Used for the diagonal (elementwise) step
// bounds of the inequality slack and multipliers, 4^d entries (d <= 13 keeps
// this below 1 GiB per vector).
void tt_full_device(const TT& v, DevBuf& out, DevBuf& tmp, Ctx& c) {
  TT_REQUIRE(v.d <= 13, "dense evaluation limited to d <= 13");
  const long m = (long)v.mo * v.mi;
  long rows = m;
  out.reserve((size_t)m * v.r[1]);
  TT_HIP(hipMemcpyAsync(out.get(), v.core(0), sizeof(double) * m * v.r[1], hipMemcpyDeviceToDevice, c.s));
  for (int k = 1; k < v.d; ++k) {
    const int rk = v.r[k], rn = v.r[k + 1];
    tmp.reserve((size_t)rows * m * rn);
    gemm(gemm_nn((int)rows, (int)(m * rn), rk, out.get(), rk, v.core(k), m * rn, tmp.get(), m * rn), c.s, &c.ws,
         GemmPrec::F64);
    std::swap(out, tmp);
    rows *= m;
  }
}

// largest |v| on the mask (per block)
__global__ void masked_absmax_kernel(const double* v, const double* mask, long n, double* part) {
  __shared__ double red[256];
  double best = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (mask[i] > 0.5) best = fmax(best, fabs(v[i]));
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// smallest ratio max(v, 0) / -dv over the masked entries with dv < 0 whose
// |v| is above the floor (per block)
__global__ void ratio_min_kernel(const double* v, const double* dv, const double* mask, long n, double floor_v,
                                 double* part) {
  __shared__ double red[256];
  double best = 1e300;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (mask[i] > 0.5 && dv[i] < 0.0 && fabs(v[i]) > floor_v) best = fmin(best, fmax(v[i], 0.0) / -dv[i]);
  red[threadIdx.x] = best;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// largest alpha with v + alpha dv >= 0 on the entries where mask = 1 (Sec. 3.4:
// the smallest eigenvalue of the diagonal pencil is the smallest entry ratio).
// Precision floor (Sec. 3.4, last paragraph): an entry whose value is below
// the precision of the TT arithmetic (64 eps of the largest masked |v|) is
// indistinguishable from the zero entries that no inequality involves, so it
// does not limit the step.
double ratio_step(const TT& v, const TT& dv, const TT& mask, Ctx& c) {
  DevBuf a, b, m, tmp;
  tt_full_device(v, a, tmp, c);
  tt_full_device(dv, b, tmp, c);
  tt_full_device(mask, m, tmp, c);
  long n = 1;
  for (int k = 0; k < v.d; ++k) n *= (long)v.mo * v.mi;
  const int nb = 256;
  DevBuf part(nb);
  std::vector<double> h(nb);
  hipLaunchKernelGGL(masked_absmax_kernel, dim3(nb), dim3(256), 0, c.s, a.get(), m.get(), n, part.get());
  TT_HIP(hipGetLastError());
  TT_HIP(hipMemcpyAsync(h.data(), part.get(), sizeof(double) * nb, hipMemcpyDeviceToHost, c.s));
  c.sync();
  double vmax = 0.0;
  for (double x : h) vmax = std::max(vmax, x);
  const double floor_v = 64.0 * 2.220446049250313e-16 * vmax;
  hipLaunchKernelGGL(ratio_min_kernel, dim3(nb), dim3(256), 0, c.s, a.get(), b.get(), m.get(), n, floor_v,
                     part.get());
  TT_HIP(hipGetLastError());
  TT_HIP(hipMemcpyAsync(h.data(), part.get(), sizeof(double) * nb, hipMemcpyDeviceToHost, c.s));
  c.sync();
  double best = 1e300;
  for (double x : h) best = std::min(best, x);
  return std::min(best, kNoBound);
}

}  // namespace

double step_length(const TT& M, const TT& dM, BlockTT& E, bool& have_E, const ttipm_params& prm,
                   unsigned long long seed, Ctx& c) {
  const double lam = min_gen_eig(M, dM, E, have_E, std::max(1, prm.eig_rank), std::max(1, prm.eig_sweeps),
                                 std::max(0, prm.eig_kick), seed, c);
  // Thm. 1: the largest alpha with M + alpha dM positive definite is -1/lambda_min
  // when lambda_min < 0 and unbounded otherwise (reported as kNoBound).
  if (!(lam < 0.0)) return kNoBound;
  return std::min(kNoBound, -1.0 / lam);
}

// ---------------------------------------------------------------------------
// the IPM iteration
// ---------------------------------------------------------------------------
// s(X) = s (B_ineq - A_ineq X): the inequality slack (>= 0 at feasible X)
TT ineq_slack(const Problem& P, const TT& X, bool homogeneous, Ctx& c) {
  TT AX = tt_matvec(P.Aineq, X, c);
  if (homogeneous) {
    tt_scale(AX, -P.sense, c);
    return AX;
  }
  return tt_add({&P.Bineq, &AX}, {P.sense, -P.sense}, c);
}

// mu = (<X, Z> + <T, s(X)>) / (n + q)  (Sec. 3.2)
// Measures of the iterate (X, Y, Z, T): objectives, residual norms, the
// complementarity <X, Z> (+ <T, slack(X)>) and mu = that / (n + q).
void iterate_measures(const Problem& P, const TT& X, const TT& Y, const TT& Z, const TT* T, ttipm_step_info& info,
                      Ctx& c) {
  double xz = tt_dot(X, Z, c);
  if (P.ineq) {
    TT sx = ineq_slack(P, X, false, c);
    xz += tt_dot(*T, sx, c);
  }
  const double mu = xz / (P.n + P.q);
  TT AY = tt_matvec(P.AeqT, Y, c);
  TT Rd = tt_add({&Z, &P.C, &AY}, {1.0, 1.0, -1.0}, c);
  TT AX = tt_matvec(P.Aeq, X, c);
  TT Rp = tt_add({&P.Beq, &AX}, {1.0, -1.0}, c);
  const double pobj = tt_dot(P.C, X, c);
  const double dobj = tt_dot(P.Beq, Y, c);
  info.mu = mu;
  info.xz = xz;
  info.pobj = pobj;
  info.dobj = dobj;
  info.norm_rp = tt_norm(Rp, c);
  info.eps_p = info.norm_rp / (1.0 + P.normB);
  double rdn2 = tt_dot(Rd, Rd, c);
  if (P.ineq) {
    TT AT = tt_matvec(P.AineqT, *T, c);
    TT Rd2 = tt_add({&Rd, &AT}, {1.0, -P.sense}, c);
    rdn2 = tt_dot(Rd2, Rd2, c);
  }
  info.norm_rd = std::sqrt(std::max(rdn2, 0.0));
  info.eps_d = info.norm_rd / (1.0 + P.normC);
  info.rel_gap = std::fabs(pobj - dobj) / (1.0 + std::fabs(pobj) + std::fabs(dobj));
  info.eps_c = mu / (1.0 + std::fabs(pobj));
  info.rank_x = X.max_rank();
  info.rank_y = Y.max_rank();
  info.rank_z = Z.max_rank();
}

void ipm_measures(const Problem& P, const State& S, ttipm_step_info& info, Ctx& c) {
  iterate_measures(P, S.X, S.Y, S.Z, P.ineq ? &S.T : nullptr, info, c);
}

bool ipm_relative_done(const ttipm_step_info& m, const ttipm_params& prm) {
  return m.rel_gap <= prm.stop_gap && m.eps_p <= 2 * prm.stop_gap && m.eps_d <= 2 * prm.stop_gap;
}

bool ipm_absolute_done(const ttipm_step_info& m, const ttipm_params& prm) {
  return m.norm_rp < prm.finish_abs && m.norm_rd < prm.finish_abs && m.xz < prm.finish_abs;
}

// Psi = ||R_p|| + ||R_d|| + mu of an iterate (the residual measure watched by the
// windowed control).  Reading: the complementarity block of R_mu enters through
// mu; its exact norm needs the rank-product TT X Z, which is never formed.
double residual_measure(const Problem& P, const TT& X, const TT& Y, const TT& Z, const TT* T, Ctx& c) {
  TT AY = tt_matvec(P.AeqT, Y, c);
  TT Rd = tt_add({&Z, &P.C, &AY}, {1.0, 1.0, -1.0}, c);
  if (P.ineq) {
    TT AT = tt_matvec(P.AineqT, *T, c);
    Rd = tt_add({&Rd, &AT}, {1.0, -P.sense}, c);
  }
  TT AX = tt_matvec(P.Aeq, X, c);
  TT Rp = tt_add({&P.Beq, &AX}, {1.0, -1.0}, c);
  double xz = tt_dot(X, Z, c);
  if (P.ineq) {
    TT sx = ineq_slack(P, X, false, c);
    xz += tt_dot(*T, sx, c);
  }
  return tt_norm(Rp, c) + tt_norm(Rd, c) + xz / (P.n + P.q);
}

namespace {

// L_Z = I kron Z + Z kron I (AHO) or Z kron I (XZ); L_X = I kron X + X kron I
// (AHO) or I kron X (XZ)
TT L_op(const Problem& P, const TT& Mv, bool aho, bool left_identity, Ctx& c) {
  TT Mm = tt_as_matrix(Mv, 2, c);
  if (aho) {
    TT a = tt_kron(P.I2, Mm, c), b = tt_kron(Mm, P.I2, c);
    return tt_add({&a, &b}, {1.0, 1.0}, c);
  }
  return left_identity ? tt_kron(P.I2, Mm, c) : tt_kron(Mm, P.I2, c);
}

// The Newton system with the multiplier updates dY and dT stored in one padded
// block dL (Sec. 3.5, Combined Multiplier Storage; masks disjoint): the dual
// column becomes -(A_eq^T P_Y + s A_ineq^T P_T) dL, the two multiplier rows
// become -(P_Y A_eq + s P_T T A_ineq) dX + (P_Y K_Y P_Y + P_T (D_ineq + K_T) P_T) dL
// with right-hand side P_Y R_p + P_T R_t, and the dX, dZ rows are unchanged.
// The operators of the block are built once per iteration (ops); the masked
// right-hand-side terms per solve, their operators kept in `store`.
struct CombinedOps {
  TT Aeq, AeqT, KY;
};

CombinedOps combined_ops(const Problem& P, const TT& TA, const TT& DK, double tol, Ctx& c) {
  CombinedOps o;
  const double s = P.sense;
  TT a1 = tt_matmat(P.PY, P.Aeq, c), a2 = tt_matmat(P.PT, TA, c);
  o.Aeq = tt_add({&a1, &a2}, {1.0, s}, c);
  TT b1 = tt_matmat(P.AeqT, P.PY, c), b2 = tt_matmat(P.AineqT, P.PT, c);
  o.AeqT = tt_add({&b1, &b2}, {1.0, s}, c);
  TT k1 = tt_matmat(P.PY, P.KY, c), k2 = tt_matmat(P.PT, DK, c);
  TT k1p = tt_matmat(k1, P.PY, c), k2p = tt_matmat(k2, P.PT, c);
  o.KY = tt_add({&k1p, &k2p}, {1.0, 1.0}, c);
  tt_round_abs(o.Aeq, tol, 1 << 30, c);
  tt_round_abs(o.AeqT, tol, 1 << 30, c);
  tt_round_abs(o.KY, tol, 1 << 30, c);
  return o;
}

NewtonSys combined_system(const NewtonSys& s0, const Problem& P, const CombinedOps& co, std::deque<TT>& store,
                          double tol, Ctx& c) {
  NewtonSys sc;
  sc.ineq = false;
  sc.sense = 1.0;
  for (int o = 0; o < OP_COUNT; ++o) sc.ops[o] = nullptr;
  sc.ops[OP_AEQ] = &co.Aeq;
  sc.ops[OP_AEQT] = &co.AeqT;
  sc.ops[OP_KY] = &co.KY;
  sc.ops[OP_LZ] = s0.ops[OP_LZ];
  sc.ops[OP_LX] = s0.ops[OP_LX];
  sc.ops[OP_EXTRA0] = s0.ops[OP_EXTRA0];
  // masked term operators in the free slots OP_EXTRA2.., one per (mask, operator)
  std::vector<std::pair<std::pair<int, int>, int>> memo;
  int next = OP_EXTRA2;
  auto masked = [&](int mask, int op) {
    for (const auto& m : memo)
      if (m.first.first == mask && m.first.second == op) return m.second;
    TT_REQUIRE(next < OP_COUNT, "combined multipliers: out of operator slots");
    const TT& M = mask == 0 ? P.PY : P.PT;
    if (op < 0) {
      store.push_back(tt_clone(M, c));
    } else {
      store.push_back(tt_matmat(M, *s0.ops[op], c));
      tt_round_abs(store.back(), tol, 1 << 30, c);
    }
    sc.ops[next] = &store.back();
    memo.push_back({{mask, op}, next});
    return next++;
  };
  // an unmasked term whose operator the combined system does not carry (A_ineq^T
  // on T in R_d) gets a slot of its own
  auto carried = [&](int op) {
    if (op < 0 || sc.ops[op] == s0.ops[op]) return op;
    for (int o = OP_EXTRA2; o < next; ++o)
      if (sc.ops[o] == s0.ops[op]) return o;
    TT_REQUIRE(next < OP_COUNT, "combined multipliers: out of operator slots");
    sc.ops[next] = s0.ops[op];
    return next++;
  };
  for (const Term& t : s0.terms) {
    if (t.res == RES_P) sc.terms.push_back({RES_P, t.coef, masked(0, t.op), t.vec});
    else if (t.res == RES_T) sc.terms.push_back({RES_P, t.coef, masked(1, t.op), t.vec});
    else sc.terms.push_back({t.res, t.coef, carried(t.op), t.vec});
  }
  return sc;
}

}  // namespace

void ipm_step(const Problem& P, State& S, const ttipm_params& prm, ttipm_step_info& info, Ctx& c,
              const ttipm_step_info* entry) {
  const double t_begin = now();
  info = entry ? *entry : ttipm_step_info{};
  info.iter = S.iter;
  if (!entry) ipm_measures(P, S, info, c);
  const double mu = info.mu;
  // Finishing phase (Sec. 3.5, Relaxing the Positive Definiteness Barrier):
  // once the relative stopping criteria hold, the iteration goes on towards
  // the absolute ones with the PD barrier relaxed to M + nu I >= 0 (nu grows
  // from 0 only after rejected updates, up to finish_nu_max), and updates are
  // accepted on a merit test.
  if (prm.finish && !S.finishing && ipm_relative_done(info, prm)) {
    S.finishing = true;
    S.nu = 0.0;
  }
  info.finishing = S.finishing ? 1 : 0;
  info.nu = S.nu;
  const double nu = S.finishing ? S.nu : 0.0;
  // the matrices whose definiteness bounds the steps: M + nu I
  TT Xb, Zb;
  if (nu > 0.0) {
    Xb = tt_add({&S.X, &P.Ivec}, {1.0, nu}, c);
    Zb = tt_add({&S.Z, &P.Ivec}, {1.0, nu}, c);
  }
  const TT& Xs = nu > 0.0 ? Xb : S.X;
  const TT& Zs = nu > 0.0 ? Zb : S.Z;
  // XZ warm-up iterations (Sec. 5.1), then AHO.  With inequality constraints the
  // warm-up is skipped (reading): the nonsymmetric XZ direction breaks the
  // symmetry of X against the mirrored multipliers T, and the iteration stalls
  // (observed identically with exact dense Newton directions).
  bool aho = S.iter >= prm.n_xz || P.ineq;
  info.direction = aho ? TTIPM_DIR_AHO : TTIPM_DIR_XZ;
  const double tolp = S.eta * (1.0 + P.normB) / 10.0;
  const double told = S.eta * (1.0 + P.normC) / 10.0;
  // operators L_Z, L_X (Sec. 3.3) rounded at the primal/dual tolerances (Sec. 3.5)
  TT LZ, LX;
  auto build_L = [&](bool use_aho) {
    const double t0 = now();
    // reading: L_Z and L_X are rounded with the Cor. 1 shift (S = I kron I) so
    // that they stay positive definite when Z and X approach singularity;
    // the two are independent, one stream each
    run_concurrent(c, {[&](Ctx& cx) {
                         LZ = round_shift(L_op(P, S.Z, use_aho, false, cx), told, &P.I16, 1 << 30, cx, nullptr);
                       },
                       [&](Ctx& cx) {
                         LX = round_shift(L_op(P, S.X, use_aho, true, cx), tolp, &P.I16, 1 << 30, cx, nullptr);
                       }});
    info.t_round += now() - t0;
  };
  build_L(aho);
  NewtonSys sys;
  sys.ineq = P.ineq;
  sys.sense = P.sense;
  sys.ops[OP_AEQ] = &P.Aeq;
  sys.ops[OP_AEQT] = &P.AeqT;
  sys.ops[OP_KY] = &P.KY;
  sys.ops[OP_LZ] = &LZ;
  sys.ops[OP_LX] = &LX;
  TT TA, DK;
  if (P.ineq) {
    TT Tdiag = tt_diag(S.T, c);
    TA = tt_matmat(Tdiag, P.Aineq, c);
    tt_round_abs(TA, told, 1 << 30, c);
    // D_ineq(X) = diag_TT(s(X)), s(X) = s (B_ineq - A_ineq X) (>=: A_ineq X - B_ineq)
    TT AX = tt_matvec(P.Aineq, S.X, c);
    TT sx = tt_add({&P.Bineq, &AX}, {P.sense, -P.sense}, c);
    tt_round_abs(sx, tolp, 1 << 30, c);
    TT Dx = tt_diag(sx, c);
    DK = tt_add({&Dx, &P.KT}, {1.0, 1.0}, c);
    tt_round_abs(DK, tolp, 1 << 30, c);
    sys.ops[OP_TA] = &TA;
    sys.ops[OP_DK] = &DK;
    sys.ops[OP_AIT] = &P.AineqT;
  }
  // combined multiplier storage (Sec. 3.5) when the masks are disjoint
  const bool comb = P.ineq && P.masks_disjoint && prm.combine_multipliers != 0;
  CombinedOps cops;
  if (comb) cops = combined_ops(P, TA, DK, told, c);
  std::deque<TT> cstore;
  NewtonSys sysc;
  // the system the AMEn solves: the combined one is rebuilt from sys's terms
  auto solve_sys = [&]() -> const NewtonSys& {
    if (!comb) return sys;
    cstore.clear();
    sysc = combined_system(sys, P, cops, cstore, told, c);
    return sysc;
  };
  // residual terms: R_d = Z + C - Aeq^T Y (- s Aineq^T T), R_p = B - Aeq X,
  // R_t = T o s(X) - mu 1_T = -s diag(T) A_ineq X (+ s diag(T) B_ineq) - mu 1_T
  //
  // Zero blocks (Sec. 3.5): a feasibility residual that already meets its
  // stopping threshold (relative 2 stop_gap; in the finishing phase the
  // absolute target) is set to zero in the Newton system, so its terms are
  // neither projected nor contracted.
  const bool zero_p = S.finishing ? info.norm_rp < prm.finish_abs : info.eps_p <= 2.0 * prm.stop_gap;
  const bool zero_d = S.finishing ? info.norm_rd < prm.finish_abs : info.eps_d <= 2.0 * prm.stop_gap;
  std::vector<Term> base;
  if (!zero_d) {
    base.push_back({RES_D, 1.0, -1, &S.Z});
    base.push_back({RES_D, 1.0, -1, &P.C});
    base.push_back({RES_D, -1.0, OP_AEQT, &S.Y});
    if (P.ineq) base.push_back({RES_D, -P.sense, OP_AIT, &S.T});
  }
  if (!zero_p) {
    base.push_back({RES_P, 1.0, -1, &P.Beq});
    base.push_back({RES_P, -1.0, OP_AEQ, &S.X});
  }
  if (P.ineq) base.push_back({RES_T, -P.sense, OP_TA, &S.X});
  if (!S.has_W) {
    S.W = block_from_frame(P.Ivec, comb ? 3 : sys.Lp(), c);
    S.has_W = true;
  }
  AmenParams ap;
  ap.tol = std::max(S.eta / 2.0, 1e-13);
  ap.max_sweeps = prm.amen_sweeps;
  ap.rank_cap = prm.rank_cap;
  ap.direct_max = prm.direct_max;
  ap.gmres_restart = prm.gmres_restart;
  ap.gmres_maxit = prm.gmres_maxit;
  ap.precond = prm.precond;
  ap.mixed = prm.precision == TTIPM_MIXED;
  // Enrichment lets the frame ranks grow past a block-ALS fixed point; it
  // fills capacity left under the rank cap.  Random directions are switched
  // off for the rest of the solve once a Newton frame has been truncated by
  // the cap, where they would only perturb the truncated solve; residual
  // directions stay on wherever a split leaves capacity.
  ap.enrich = prm.enrich;
  ap.global_stop = prm.amen_global_stop;
  ap.kick = (prm.enrich == 0 && S.frame_capped) ? 0 : std::max(0, prm.kick);
  ap.verbose = prm.verbose;
  ap.kick_sweeps = std::max(0, prm.kick_sweeps);
  ap.mlp = prm.mlp ? &const_cast<tt_mlp*>(static_cast<const tt_mlp*>(prm.mlp))->net : nullptr;
  ap.collect_probes = std::max(0, prm.collect_probes);
  ap.collect_cap = (long)prm.collect_cap;
  ap.mu = std::max(mu, 1e-300);
  ap.seed = S.seed + 31ull * (unsigned long long)S.iter;
  // --- predictor: affine direction (target mu = 0) ---
  const int L = comb ? 2 : sys.L();   // solved components; dZ is component L
  // components of the direction: dX = 0, dZ = L; dY = 1 and dT = 2, or with
  // combined storage dY = P_Y dL and dT = P_T dL with dL = 1
  auto comp_y = [&]() {
    if (!comb) return S.W.component(1, c);
    TT dl = S.W.component(1, c);
    return tt_matvec(P.PY, dl, c);
  };
  auto comp_t = [&]() {
    if (!comb) return S.W.component(2, c);
    TT dl = S.W.component(1, c);
    TT t = tt_matvec(P.PT, dl, c);
    tt_round_abs(t, 1e-14 * std::max(tt_norm(t, c), 1e-300), 1 << 30, c);
    return t;
  };
  const unsigned long long sd = S.seed + 7919ull * (unsigned long long)S.iter;
  AmenInfo ai_p;
  TT dX, dZ, dT, sx, dsx;
  double a_p = 0.0, a_d = 0.0;
  auto predictor = [&]() {
    sys.terms = base;
    sys.terms.push_back({RES_C, 1.0, OP_LZ, &S.X});   // (R_t keeps its mu term only in the corrector)
    ai_p = AmenInfo{};
    amen_solve(solve_sys(), S.W, ap, ai_p, c);
    S.frame_capped |= ai_p.capped;
    dX = S.W.component(0, c);
    dZ = S.W.component(L, c);
    const double t1 = now();
    // affine (predictor) steps: the full Thm. 1 step, clipped to 1; with
    // inequalities also s(X + a_p dX) >= 0 and T + a_d dT >= 0 on the active
    // mask (Sec. 3.4: the diagonal pencils reduce to entry ratios)
    // the primal and dual eigen-solves are independent: one stream each
    run_concurrent(c, {[&](Ctx& cx) { a_p = std::min(1.0, step_length(Xs, dX, S.EX, S.has_EX, prm, sd + 1, cx)); },
                       [&](Ctx& cx) { a_d = std::min(1.0, step_length(Zs, dZ, S.EZ, S.has_EZ, prm, sd + 2, cx)); }});
    if (P.ineq) {
      dT = comp_t();
      sx = ineq_slack(P, S.X, false, c);
      dsx = ineq_slack(P, dX, true, c);
      a_p = std::min(a_p, ratio_step(sx, dsx, P.oneT, c));
      a_d = std::min(a_d, ratio_step(S.T, dT, P.oneT, c));
    }
    info.t_step += now() - t1;
  };
  predictor();
  // AHO -> XZ fallback (Sec. 3.5): when the AHO solve misses its residual
  // target with the rank cap binding, or admits almost no step, the
  // iteration is redone with the XZ direction, which often needs lower TT
  // ranks.  Not with inequalities (reading: XZ breaks the symmetry of X
  // against the mirrored multipliers there).
  if (aho && !P.ineq && prm.xz_fallback &&
      ((ai_p.capped && ai_p.last_max_res > ap.tol) || std::max(a_p, a_d) < 1e-3)) {
    aho = false;
    info.direction = TTIPM_DIR_XZ;
    info.xz_fallback = 1;
    build_L(false);
    predictor();
  }
  const double coef = aho ? 2.0 : 1.0;
  double t1 = 0.0;
  // mu_aff = (<X + a_p dX, Z + a_d dZ> + <T + a_d dT, s(X + a_p dX)>) / (n + q)
  const double xz = tt_dot(S.X, S.Z, c), xdz = tt_dot(S.X, dZ, c), dxz = tt_dot(dX, S.Z, c),
               dxdz = tt_dot(dX, dZ, c);
  double ts_aff = 0.0;
  if (P.ineq)
    ts_aff = tt_dot(S.T, sx, c) + a_p * tt_dot(S.T, dsx, c) + a_d * tt_dot(dT, sx, c) +
             a_p * a_d * tt_dot(dT, dsx, c);
  const double mu_aff = (xz + a_d * xdz + a_p * dxz + a_p * a_d * dxdz + ts_aff) / (P.n + P.q);
  const double sigma = std::pow(std::max(mu_aff, 0.0) / mu, 3.0);
  // --- corrector: centring and the second-order term L_{dZ_aff} vec dX_aff ---
  TT LdZ, LdX_unused;
  {
    TT dZm = tt_as_matrix(dZ, 2, c);
    if (aho) {
      TT a = tt_kron(P.I2, dZm, c), b = tt_kron(dZm, P.I2, c);
      LdZ = tt_add({&a, &b}, {1.0, 1.0}, c);
    } else {
      LdZ = tt_kron(dZm, P.I2, c);
    }
    tt_round_abs(LdZ, told, 1 << 30, c);
  }
  sys.ops[OP_EXTRA0] = &LdZ;
  sys.terms = base;
  sys.terms.push_back({RES_C, 1.0, OP_LZ, &S.X});
  sys.terms.push_back({RES_C, 1.0, OP_EXTRA0, &dX});
  sys.terms.push_back({RES_C, -coef * sigma * mu, -1, &P.Ivec});
  TT dTdiag;
  if (P.ineq) {
    sys.terms.push_back({RES_T, -sigma * mu, -1, &P.oneT});
    // second-order term of R_t: dT_aff o ds_aff
    dTdiag = tt_diag(dT, c);
    tt_round_abs(dTdiag, told, 1 << 30, c);
    sys.ops[OP_EXTRA1] = &dTdiag;
    sys.terms.push_back({RES_T, 1.0, OP_EXTRA1, &dsx});
  }
  AmenInfo ai_c;
  const NewtonSys& sys_c = solve_sys();
  amen_solve(sys_c, S.W, ap, ai_c, c);
  S.frame_capped |= ai_c.capped;
  // Global FP64 residual of the corrector system (Sec. 3.3, Lemma "AMEn
  // Directions as Inexact Newton Directions": ||K dU + R|| <= eta ||R||).  In
  // mixed precision a direction that misses it is refined by FP64 AMEn
  // sweeps warm-started from it (iterative refinement of the Newton solve).
  if (prm.newton_check) {
    const double t0 = now();
    double res = 0.0, rhs = 0.0;
    if (ai_c.newton_res_final) {
      info.newton_res = ai_c.newton_res;   // the AMEn stopping rule evaluated this direction already
    } else {
      newton_residual(sys_c, S.W, &res, &rhs, c);
      info.newton_res = rhs > 0 ? res / rhs : (res < 0 ? -1.0 : 0.0);
    }
    if (ap.mixed && info.newton_res > S.eta) {
      AmenParams ar = ap;
      ar.mixed = false;
      ar.max_sweeps = std::max(2, prm.refine_sweeps);
      AmenInfo ai_r;
      amen_solve(sys_c, S.W, ar, ai_r, c);
      S.frame_capped |= ai_r.capped;
      info.refine_sweeps = ai_r.sweeps;
      ai_c.krylov_iters += ai_r.krylov_iters;
      ai_c.t_env += ai_r.t_env;
      ai_c.t_solve += ai_r.t_solve;
      ai_c.t_svd += ai_r.t_svd;
      newton_residual(sys_c, S.W, &res, &rhs, c);
      info.newton_res = rhs > 0 ? res / rhs : (res < 0 ? -1.0 : 0.0);
    }
    info.t_check = now() - t0;
  }
  TT dX2 = S.W.component(0, c), dY2 = comp_y(), dZ2 = S.W.component(L, c);
  TT dT2;
  if (P.ineq) dT2 = comp_t();
  t1 = now();
  run_concurrent(c, {[&](Ctx& cx) { info.alpha_p_max = step_length(Xs, dX2, S.EX, S.has_EX, prm, sd + 3, cx); },
                     [&](Ctx& cx) { info.alpha_d_max = step_length(Zs, dZ2, S.EZ, S.has_EZ, prm, sd + 4, cx); }});
  if (P.ineq) {
    TT ds2 = ineq_slack(P, dX2, true, c);
    info.alpha_p_max = std::min(info.alpha_p_max, ratio_step(sx, ds2, P.oneT, c));
    info.alpha_d_max = std::min(info.alpha_d_max, ratio_step(S.T, dT2, P.oneT, c));
  }
  a_p = std::min(1.0, prm.tau * info.alpha_p_max);
  a_d = std::min(1.0, prm.tau * info.alpha_d_max);
  info.t_step += now() - t1;
  // --- update and rounding with spectral shift (Cor. 1) ---
  // Safeguard (Sec. 3.3, damped retry): the TT eigen-solver bounds lambda_min
  // from above, so the step can overshoot; the updated X and Z are checked
  // with a DMRG estimate of lambda_min against the identity, and a step whose
  // estimate is not positive is halved and retried.
  //
  // Windowed residual control (Sec. 3.3, condition (G4) of the safeguarded
  // TT-IPM theorem): the residual measure Psi of the rounded, shifted update is
  // compared with the largest Psi of the last M + 1 accepted iterates; a step
  // that exceeds it by more than the rounding budget of the update is damped
  // (both step lengths halved) and retried.
  t1 = now();
  const int cap = prm.iter_rank_cap > 0 ? prm.iter_rank_cap : 4 * prm.rank_cap;
  {
    auto pd_min = [&](const TT& M, BlockTT& E, bool& have, Ctx& cx) {
      return min_gen_eig(P.Ivec, M, E, have, std::max(1, prm.eig_rank), std::max(1, prm.eig_sweeps),
                         std::max(0, prm.eig_kick), sd + 11, cx);
    };
    const int M = std::max(0, prm.g4_window);
    const double psi_k = info.eps_p * (1.0 + P.normB) + info.eps_d * (1.0 + P.normC) + mu;
    S.psi_hist.push_back(psi_k);
    while ((int)S.psi_hist.size() > M + 1) S.psi_hist.erase(S.psi_hist.begin());
    const double theta = *std::max_element(S.psi_hist.begin(), S.psi_hist.end());
    // reading: the control applies once the XZ warm-up is over and the window
    // is full ("for all sufficiently large k" in (G4)); the allowed perturbation
    // is the Cor. 1 budget of the X and Z roundings
    const bool g4_on = M > 0 && S.iter >= prm.n_xz && (int)S.psi_hist.size() == M + 1;
    const double rho = tolp + told;
    struct Trial {
      TT X, Y, Z, T;
      double a_p = 0, a_d = 0, psi = 0;
      ShiftInfo sx, sz;
      int bt = 0;
    };
    // X + a_p dX and Z + a_d dZ: rounding, shift and safeguard, one stream each
    // (the dual step a_d is final once the Z branch ends, so Y follows it)
    auto attempt = [&](double ap, double ad) {
      Trial t;
      int bt_p = 0, bt_d = 0;
      auto primal = [&](Ctx& cx) {
        for (int tries = 0;; ++tries) {
          if (tries > 6) {           // no acceptable step: keep the iterate
            ap = 0.0;
            t.X = tt_clone(S.X, cx);
            t.sx = ShiftInfo{};
            break;
          }
          TT Xs = tt_add({&S.X, &dX2}, {1.0, ap}, cx);
          t.X = round_shift(std::move(Xs), tolp, &P.Ivec, cap, cx, &t.sx, prm.shift_mode != 0);
          if (pd_min(t.X, S.EXc, S.has_EXc, cx) > -nu) break;
          ap *= 0.5;
          bt_p++;
        }
      };
      auto dual = [&](Ctx& cx) {
        for (int tries = 0;; ++tries) {
          if (tries > 6) {
            ad = 0.0;
            t.Z = tt_clone(S.Z, cx);
            t.sz = ShiftInfo{};
            break;
          }
          TT Zs = tt_add({&S.Z, &dZ2}, {1.0, ad}, cx);
          t.Z = round_shift(std::move(Zs), told, &P.Ivec, cap, cx, &t.sz, prm.shift_mode != 0);
          if (pd_min(t.Z, S.EZc, S.has_EZc, cx) > -nu) break;
          ad *= 0.5;
          bt_d++;
        }
        TT Yn = tt_add({&S.Y, &dY2}, {1.0, ad}, cx);
        t.Y = round_shift(std::move(Yn), told, nullptr, cap, cx, nullptr);
      };
      run_concurrent(c, {primal, dual});
      if (P.ineq) {
        TT Tn = tt_add({&S.T, &dT2}, {1.0, ad}, c);
        t.T = round_shift(std::move(Tn), told, &P.oneT, cap, c, nullptr, prm.shift_mode != 0);
      }
      t.a_p = ap;
      t.a_d = ad;
      t.bt = bt_p + bt_d;
      return t;
    };
    Trial best;
    bool have_best = false;
    const double a_p0 = a_p, a_d0 = a_d;
    if (S.finishing) {
      // merit acceptance: the merit ||R_p|| + ||R_d|| + |<X, Z>| (the
      // quantities of the absolute criteria) must decrease while neither
      // residual rises above max(current, its absolute target) and eps_p,
      // eps_d and the gap stay within max(current, the relative stopping
      // bound), so that every accepted iterate still meets the relative
      // criteria; damped retries, else the iterate is kept
      const double phi0 = info.norm_rp + info.norm_rd + std::fabs(info.xz);
      const double lim_p = std::max(info.eps_p, 2.0 * prm.stop_gap), lim_d = std::max(info.eps_d, 2.0 * prm.stop_gap);
      const double lim_g = std::max(info.rel_gap, prm.stop_gap);
      const double lim_rp = std::max(info.norm_rp, prm.finish_abs), lim_rd = std::max(info.norm_rd, prm.finish_abs);
      bool accepted = false;
      for (int g = 0;; ++g) {
        Trial t = attempt(a_p, a_d);
        info.backtracks += t.bt;
        ttipm_step_info tm{};
        iterate_measures(P, t.X, t.Y, t.Z, P.ineq ? &t.T : nullptr, tm, c);
        t.psi = tm.norm_rp + tm.norm_rd + std::fabs(tm.xz);
        if (t.psi < phi0 && tm.eps_p <= lim_p && tm.eps_d <= lim_d && tm.rel_gap <= lim_g && tm.norm_rp <= lim_rp &&
            tm.norm_rd <= lim_rd && (t.a_p > 0.0 || t.a_d > 0.0)) {
          best = std::move(t);
          accepted = true;
          break;
        }
        const double ap_next = 0.5 * t.a_p, ad_next = 0.5 * t.a_d;
        if (g >= std::max(0, prm.g4_retries) || (ap_next == 0.0 && ad_next == 0.0)) break;
        info.g4_retries++;
        a_p = ap_next;
        a_d = ad_next;
      }
      if (!accepted) {
        best = Trial{};
        best.X = tt_clone(S.X, c);
        best.Y = tt_clone(S.Y, c);
        best.Z = tt_clone(S.Z, c);
        if (P.ineq) best.T = tt_clone(S.T, c);
        best.a_p = best.a_d = 0.0;
        // the direction is recomputed next iteration: with a more relaxed
        // barrier when the PD bounds held the step short, and in every case
        // with a tenfold tighter forcing term (solve and rounding tolerances)
        if (std::min(a_p0, a_d0) < 0.1) S.nu = std::min(std::max(10.0 * S.nu, 1e-7), prm.finish_nu_max);
        S.eta = std::max(0.1 * S.eta, 1e-12);
        info.finish_rejected = 1;
      }
      have_best = true;
    }
    for (int g = 0; !have_best; ++g) {
      Trial t = attempt(a_p, a_d);
      info.backtracks += t.bt;
      if (!g4_on) {
        best = std::move(t);
        break;
      }
      t.psi = residual_measure(P, t.X, t.Y, t.Z, P.ineq ? &t.T : nullptr, c);
      const bool ok = t.psi <= theta + rho;
      const double ap_next = 0.5 * t.a_p, ad_next = 0.5 * t.a_d;
      if (!have_best || t.psi < best.psi) {
        best = std::move(t);
        have_best = true;
      }
      // after the last damping the trial with the smallest Psi is taken, so
      // that the iteration never stands still on a repeated direction
      if (ok || g >= std::max(0, prm.g4_retries) || (ap_next == 0.0 && ad_next == 0.0)) break;
      info.g4_retries++;
      a_p = ap_next;
      a_d = ad_next;
    }
    a_p = best.a_p;
    a_d = best.a_d;
    info.psi = (g4_on || S.finishing) ? best.psi : psi_k;
    info.zeta_x = best.sx.zeta;
    info.zeta_x_cap = std::sqrt(std::max(0.0, best.sx.zeta * best.sx.zeta - best.sx.zeta_tol * best.sx.zeta_tol));
    info.zeta_z = best.sz.zeta;
    info.zeta_z_cap = std::sqrt(std::max(0.0, best.sz.zeta * best.sz.zeta - best.sz.zeta_tol * best.sz.zeta_tol));
    S.X = std::move(best.X);
    S.Z = std::move(best.Z);
    S.Y = std::move(best.Y);
    if (P.ineq) S.T = std::move(best.T);
    S.dX = tt_clone(dX2, c);
    S.dY = tt_clone(dY2, c);
    S.dZ = tt_clone(dZ2, c);
    if (P.ineq) S.dT = tt_clone(dT2, c);
  }
  info.t_round += now() - t1;
  info.alpha_p = a_p;
  info.alpha_d = a_d;
  info.sigma = sigma;
  info.eta = S.eta;
  info.sweeps_pred = ai_p.sweeps;
  info.sweeps_corr = ai_c.sweeps;
  info.krylov_iters = ai_p.krylov_iters + ai_c.krylov_iters;
  info.mlp_used = ai_p.mlp_used + ai_c.mlp_used;
  info.mlp_fallbacks = ai_p.mlp_fallbacks + ai_c.mlp_fallbacks;
  info.rank_w = std::max(ai_p.max_rank, ai_c.max_rank);
  info.t_check += ai_p.t_check + ai_c.t_check;
  info.t_env = ai_p.t_env + ai_c.t_env;
  info.t_solve = ai_p.t_solve + ai_c.t_solve;
  info.t_svd = ai_p.t_svd + ai_c.t_svd;
  // in the finishing phase the floor delta of the forcing term gives way to
  // one that keeps the rounding tolerances (eta (1 + ||b||) / 10, eta (1 +
  // ||C||) / 10) below a tenth of the absolute targets
  const double floor = S.finishing ? std::min(prm.delta, prm.finish_abs / (1.0 + std::max(P.normB, P.normC)))
                                   : prm.delta;
  S.eta = std::max(std::min(S.eta, prm.cmu * mu), std::min(floor, S.eta));
  S.iter += 1;
  info.t_total = now() - t_begin;
}

}  // namespace ttipm
