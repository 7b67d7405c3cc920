// Device-resident tensor trains and the TT algebra of the paper (Sec. 2.3,
// Sec. 3.1, Sec. 3.3): sums by core concatenation, scaling, per-core
// Kronecker products, diag_TT, TT matrix-vector products, inner products,
// environments (interfaces), projected local products and rounding.
#pragma once

#include <functional>
#include <vector>

#include "common.hpp"
#include "gemm.hpp"

namespace ttipm {

// A tensor train with uniform modes: core k is [r[k]][mo][mi][r[k+1]] (mi = 1 for vectors).
struct TT {
  int d = 0, mo = 4, mi = 1;
  std::vector<int> r;
  std::vector<DevBuf> cores;

  TT() = default;
  TT(int d_, int mo_, int mi_) : d(d_), mo(mo_), mi(mi_), r(d_ + 1, 1), cores(d_) {}
  TT(TT&&) = default;
  TT& operator=(TT&&) = default;

  long core_size(int k) const { return (long)r[k] * mo * mi * r[k + 1]; }
  int max_rank() const {
    int m = 1;
    for (int x : r) m = x > m ? x : m;
    return m;
  }
  double* core(int k) const { return cores[k].get(); }
  void alloc(int k) { cores[k].reserve((size_t)core_size(k)); }
};

// Execution context: stream, scratch buffers and the GEMM precision of contractions.
struct Ctx {
  hipStream_t s = nullptr;
  Workspace ws;               // split-K partials
  DevBuf t1, t2, t3, perm, perm2;   // contraction intermediates
  DevBuf dscr, dscr2, dscr3;  // dense factorisation scratch
  DevBuf ired;                // int scratch (status words)
  DevBuf dot_part, dot_out;
  std::vector<DevBuf> gbuf;   // per-product stage buffers of grouped local products
  std::vector<DevBuf> lbuf;   // callers' operands of grouped local products
  GemmPrec prec = GemmPrec::F64;
  double* hbuf = nullptr;     // pinned host staging
  size_t hbuf_n = 0;
  ~Ctx();
  double* host(size_t n);     // pinned host buffer of >= n doubles
  void sync() { TT_HIP(hipStreamSynchronize(s)); }
};

// Runs the tasks concurrently: the first on the calling thread with c, the
// others on threads of their own, each with a worker context (own stream and
// scratch, c's GEMM precision).  c is synchronised first and every context at
// the end; the first exception of any task is rethrown.  Tasks must not write
// shared state.
void run_concurrent(Ctx& c, const std::vector<std::function<void(Ctx&)>>& tasks);

// ---- construction and copies ---------------------------------------------
TT tt_from_host(const std::vector<std::vector<double>>& cores, const std::vector<int>& ranks, int mo, int mi,
                Ctx& c);
TT tt_from_view(const tt_view& v, Ctx& c);   // deep copy of caller buffers
TT tt_clone(const TT& a, Ctx& c);
std::vector<std::vector<double>> tt_to_host(const TT& a, Ctx& c);
// rank-1 TT with every core equal to the given mode vector/matrix (host values)
TT tt_rank1(int d, int mo, int mi, const std::vector<double>& core, Ctx& c);

// ---- algebra -----------------------------------------------------------------
TT tt_add(const std::vector<const TT*>& terms, const std::vector<double>& coef, Ctx& c);
void tt_scale(TT& a, double s, Ctx& c);
TT tt_kron(const TT& A, const TT& B, Ctx& c);          // per-core Kronecker of TT matrices
TT tt_diag(const TT& v, Ctx& c);                       // diag_TT of a TT vector
TT tt_matvec(const TT& A, const TT& x, Ctx& c);        // A x (A: mo x mi modes, x: mi modes)
TT tt_matmat(const TT& A, const TT& B, Ctx& c);        // A B
TT tt_as_matrix(const TT& v, int n, Ctx& c);           // vec_TT^{-1}: [r][n*n][r'] -> [r][n][n][r'] (copy)
TT tt_as_vector(const TT& m, Ctx& c);                  // vec_TT:  [r][n][n][r'] -> [r][n*n][r'] (copy)
TT tt_transpose(const TT& A, Ctx& c);                  // swap mode indices of a TT matrix
double tt_dot(const TT& x, const TT& y, Ctx& c);       // <x, y> (synchronises)
double tt_norm(const TT& x, Ctx& c);
double tt_sandwich(const TT& u, const TT& A, const TT& v, Ctx& c);  // u^T A v
// <Oi vi, Oj vj> for TT vectors vi, vj and operators Oi, Oj on them (nullptr =
// identity), never forming Oi vi: the norm of a sum of operator images is a
// sum of these (synchronises)
double tt_op_dot(const TT& vi, const TT* Oi, const TT& vj, const TT* Oj, Ctx& c);
// Several such inner products at once: the k-th stage of every pair runs in
// grouped launches (one sweep over the cores for all pairs, one synchronisation).
struct OpDotPair {
  const TT* vi;
  const TT* Oi;
  const TT* vj;
  const TT* Oj;
};
std::vector<double> tt_op_dots(const std::vector<OpDotPair>& pairs, Ctx& c);

// ---- environments and projected local products (Sec. 3.3) ---------------------
// phi_in/phi_out layouts as in tt_contract_interfaces; O == nullptr is the identity.
void env_left_step(const double* phi, int ra, int R, int rc, const double* V, int mo, int ra2, const double* O,
                   int Rp, int mi, const double* U, int rc2, double* out, Ctx& c);
void env_right_step(const double* phi, int ra2, int Rp, int rc2, const double* V, int mo, int ra,
                    const double* O, int R, int mi, const double* U, int rc, double* out, Ctx& c);
// Several environment steps of one direction at once (their k-th GEMMs share
// grouped launches).  The fields hold the arguments of env_left_step, or of
// env_right_step, in that function's order (for a right step: phi, ra2, Rp,
// rc2, V, mo, ra, O, R, mi, U, rc, out).  Outputs must be distinct.
struct EnvStepArgs {
  const double* phi;
  int ra, R, rc;
  const double* V;
  int mo, ra2;
  const double* O;
  int Rp, mi;
  const double* U;
  int rc2;
  double* out;
};
void env_steps(const std::vector<EnvStepArgs>& steps, bool left, Ctx& c);
// y = alpha * P x + beta * y with P the projected operator between a test
// frame (ranks r, s) and a trial TT core x [rc][m][rd]:
//   y[a][i][b] = sum phiL[a][al][c] O[al][i][j][be] x[c][j][e] phiR[b][be][e]
// Operm is O permuted to [i][be][al][j] (permute_op_core), nullptr = identity.
void local_apply(const double* phiL, int r, int R, int rc, const double* Operm, int m, const double* phiR, int s,
                 int Rp, int rd, const double* x, double* y, double alpha, double beta, Ctx& c);
// Several local_apply calls with grouped stage launches: the same result as
// calling local_apply for each element in order (outputs may repeat; the
// contributions to one output keep the list order).  Operm as local_apply.
struct LocalApplyArgs {
  const double* phiL;
  int r, R, rc;
  const double* Operm;
  int m;
  const double* phiR;
  int s, Rp, rd;
  const double* x;
  double* y;
  double alpha, beta;
};
// A bump allocator over caller-provided device memory (base == nullptr:
// count only).  Offsets are rounded to 256 bytes.
struct Arena {
  double* base = nullptr;
  size_t cap = 0, used = 0;
  double* take(size_t n) {
    const size_t off = (used + 31) & ~size_t(31);
    used = off + n;
    TT_REQUIRE(!base || used <= cap, "scratch arena overflow");
    return base ? base + off : nullptr;
  }
};
// With arena: stage buffers are taken from it and split-K partials use the
// rest of it (never grown); with dry as well nothing is launched and
// *ws_need receives the split-K partials the launches would need (a dry run
// takes operand pointers only as markers: Operm != nullptr means an operator).
void local_apply_many(const std::vector<LocalApplyArgs>& v, Ctx& c, Arena* arena = nullptr, bool dry = false,
                      size_t* ws_need = nullptr);
void permute_op_core(const double* O, int R, int m, int Rp, double* out, hipStream_t s);

// ---- orthogonalisation and rounding --------------------------------------------
// Orthonormalise the q rows (each of length len) of a row-major matrix in place (Householder QR).
void orth_rows(double* G, int q, int len, Ctx& c);
// Right-orthogonalise cores d-1 .. downto+1 (ranks may shrink).
void tt_orth_right(TT& t, int downto, Ctx& c);
// TT rounding (abs tolerance eps, per-bond eps/sqrt(d-1)); returns zeta = ||t - t~||_F.
// zeta_tol receives the part the tolerance alone discards (<= eps); the rest of
// zeta (zeta^2 - zeta_tol^2) is forced by max_rank.
double tt_round_abs(TT& t, double eps, int max_rank, Ctx& c, bool* capped = nullptr, double* zeta_tol = nullptr);

// SVD of a row-major matrix M (rows x cols) on the device: U row-major
// (rows x k), sigma (host, k values), Vt row-major (k x cols), k = min(rows, cols).
struct SvdOut {
  DevBuf U, Vt;
  std::vector<double> sigma;
  int k = 0;
};
void svd_rowmajor(const double* M, int rows, int cols, SvdOut& out, Ctx& c);
// One side only: sigma and U (left) or Vt (right), with k = min(rows, cols).
void svd_rowmajor_side(const double* M, int rows, int cols, bool left, SvdOut& out, Ctx& c);

}  // namespace ttipm
