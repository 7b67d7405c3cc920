// Block-AMEn solve of the TT Newton system (Sec. 2.3 "Block Tensor-Train",
// Sec. 3.3): one shared frame W for dX, dY, [dT], dZ; at each core the reduced
// projected system of eq. (reduced_kkt_system) is solved with dZ eliminated
// locally, the block index is moved to the neighbour by a truncated SVD, and
// the left/right environments of every operator and right-hand-side term are
// cached and updated incrementally.
#pragma once

#include <functional>

#include <string>
#include <vector>

#include "tt.hpp"

namespace ttipm {

// Indices of the system operators (all TT matrices with 4 x 4 modes).
enum SysOpId {
  OP_AEQ = 0, OP_AEQT, OP_KY, OP_LZ, OP_LX, OP_TA, OP_DK, OP_AIT,
  // operators used only by right-hand-side terms
  OP_EXTRA0, OP_EXTRA1, OP_EXTRA2, OP_EXTRA3, OP_EXTRA4, OP_EXTRA5, OP_EXTRA6, OP_EXTRA7, OP_EXTRA8, OP_EXTRA9,
  OP_COUNT
};

// Residual blocks of eq. (tt-kkt-newton-system).
enum ResId { RES_D = 0, RES_P = 1, RES_C = 2, RES_T = 3 };

// A right-hand-side term  coef * op(vec)  contributing to residual `res`
// (op < 0: the vector itself).  Residuals are never formed as TTs; their
// projections come from environments of (W | op | vec).
struct Term {
  int res;
  double coef;
  int op;
  const TT* vec;
};

struct NewtonSys {
  bool ineq = false;
  double sense = 1.0;          // +1: A_ineq X <= B_ineq; -1: >= (Sec. 4.3)
  const TT* ops[OP_COUNT] = {};
  std::vector<Term> terms;
  int L() const { return ineq ? 3 : 2; }       // solved components
  int Lp() const { return L() + 1; }           // stored components (dZ last)
};

// Shared-frame block TT; the block core at `pos` is [Lp][r_pos][4][r_pos+1].
struct BlockTT {
  int d = 0, pos = 0, Lp = 3, m = 4;   // m: mode size of every core
  std::vector<int> r;
  std::vector<DevBuf> cores;
  DevBuf blk;
  long blk_size() const { return (long)Lp * r[pos] * m * r[pos + 1]; }
  TT component(int l, Ctx& c) const;   // the TT of component l
};

// Move the block index to the right (dir > 0) or left neighbour by a truncated
// SVD of the component-normalised block core (relative tolerance, rank cap).
// kick > 0 appends that many seeded random orthonormal directions to the kept
// factor (enrichment), within the rank cap.
// G (q x len, row-major) = q seeded Gaussian rows orthonormalised against q0
// orthonormal vectors b_j (element i of b_j at B[j*bj + i*bi]; two Gram-Schmidt
// passes) and against each other (QR): the random enrichment of a TT core.
void random_orth_rows(const double* B, int q0, long bj, long bi, int len, double* G, int q, unsigned long long seed,
                      Ctx& c);
// With a candidate provider (it writes candidate rows of the kept factor's
// length, the sketched residual of the local system (see amen_solve), and
// returns their pointer and count) the kick directions are their leading
// principal directions.  Either kind fills only capacity left under the cap;
// the provider is called only when there is such capacity.
using CandidateFn = std::function<int(const double** rows)>;
bool split_block(BlockTT& W, int dir, double tol_rel, int cap, Ctx& c, int kick = 0,
                 unsigned long long seed = 0, const CandidateFn* cand = nullptr);
// Norm of a device vector (deterministic; synchronises).
double dev_norm(const double* x, long n, Ctx& c);

struct AmenParams {
  double tol = 1e-6;        // local residual target (also the SVD truncation budget / sqrt(d))
  int max_sweeps = 6;       // half-sweeps (alternating direction)
  int rank_cap = 32;
  int direct_max = 1024;    // local systems of size <= direct_max are solved densely
  int gmres_restart = 40;
  int gmres_maxit = 400;
  int precond = 0;          // TT_PREC_*
  bool mixed = false;       // BF16 MFMA contractions inside the Krylov solve
  int kick = 2;             // enrichment directions added at every block move
  int enrich = 1;           // 1: the leading directions of the sketched Newton residual (AMEn,
                            // Sec. 2.3); 0: seeded random directions
  unsigned long long seed = 0;
  int verbose = 0;          // >= 2: one line per sweep to stderr
  int kick_sweeps = 1 << 30; // enrichment only in the first kick_sweeps half-sweeps
  struct Mlp* mlp = nullptr;  // learned preconditioner (precond == TT_PREC_MLP) and dataset sink
  int collect_probes = 0;    // > 0: add every local system's blocks to mlp's dataset
  long collect_cap = 0;
  double mu = 1.0;           // barrier parameter (a context feature of the MLP)
  int global_stop = 1;       // capped solves: stop once the global Newton residual stagnates
};

struct AmenInfo {
  int sweeps = 0;
  int krylov_iters = 0;
  int max_rank = 0;
  double last_max_res = 0.0;
  bool capped = false;      // some split was limited by the rank cap (not by the tolerance)
  int mlp_used = 0, mlp_fallbacks = 0;
  double t_env = 0, t_solve = 0, t_svd = 0, t_check = 0;
  double newton_res = -1.0;  // last global ratio ||K dU + R|| / ||R|| evaluated by the stopping rule
  bool newton_res_final = false;  // ... and it is that of the returned direction
};

// Solve the Newton system starting from W, whose block sits at an end core
// (0 or d-1).  On return the block is at the end core where the last
// half-sweep left it, which is the warm start of the next call.
void amen_solve(const NewtonSys& sys, BlockTT& W, const AmenParams& prm, AmenInfo& info, Ctx& c);

// Global residual of the Newton system for the direction held in W (the
// unreduced system of eq. (tt-kkt-newton-system) with the system's own,
// rounded operators): *res = ||K dU + R||, *rhs = ||R||, summed over the
// block rows, each norm exact from operator-image inner products (no image is
// formed).  The forcing condition of Sec. 3.3 (Lemma "AMEn Directions as
// Inexact Newton Directions") asks res <= eta rhs.
// rr (optional): the right-hand-side part ||R_b||^2 of every block row, which
// does not depend on the direction; filled by the first call that gets it
// and reused by later calls for the same system.
struct ResidualRhs {
  bool have = false;
  double r2[4] = {0.0, 0.0, 0.0, 0.0};
};
void newton_residual(const NewtonSys& sys, const BlockTT& W, double* res, double* rhs, Ctx& c,
                     ResidualRhs* rr = nullptr);

// Build an initial block TT (block at 0) from a frame TT (e.g. the identity).
BlockTT block_from_frame(const TT& frame, int Lp, Ctx& c);

// ---- local systems (used by amen_solve and by the C ABI) -----------------------
// Dense projected operator [(a,i,b)][(c,j,e)] (p x p) from environments.
void local_dense_op(const double* phiL, int r, int R, const double* O, int m, const double* phiR, int s, int Rp,
                    double* out, Ctx& c);
// Several dense projected operators at once (grouped GEMM launches, one sync).
struct DenseOpArgs {
  const double* phiL;
  int r, R;
  const double* O;
  int m;
  const double* phiR;
  int s, Rp;
  double* out;
};
void local_dense_ops(const std::vector<DenseOpArgs>& v, Ctx& c);

}  // namespace ttipm
