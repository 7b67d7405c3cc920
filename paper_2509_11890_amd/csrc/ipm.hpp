// The TT primal-dual interior-point method (Alg. 1 with the TT machinery of
// Sec. 3): problem encodings of Sec. 4, the initial point of Sec. 5.1, the
// Mehrotra predictor-corrector Newton solves by block AMEn, the step length of
// Sec. 3.4, rounding with the spectral shift of Cor. 1 and the tolerance
// schedule of Sec. 3.5.
#pragma once

#include "amen.hpp"

namespace ttipm {

struct Problem {
  int kind = 0, d = 0;
  double n = 0, q = 0;
  double lam0 = 1.0;
  double x0_ineq = 0.0, t0_ineq = 1e-3;   // X0 = lam0 I + x0_ineq A_ineq(J), T0 = t0_ineq A_ineq(J)
  bool ineq = false;
  double sense = 1.0;
  TT C, Aeq, AeqT, KY, Beq;          // vec_TT vectors (mode 4) and operators (4 x 4)
  TT Aineq, AineqT, KT, Bineq, oneT;
  TT Ivec;                           // vec_TT(I)
  TT PY, PT;                         // non-idle multiplier masks I - K_Y, I - K_T (inequalities)
  bool masks_disjoint = false;       // P_Y P_T = 0: Y and T can share one padded block (Sec. 3.5)
  TT I2;                             // identity TT matrix, 2 x 2 modes
  TT I16;                            // identity operator I kron I, 4 x 4 modes
  double normB = 0, normC = 0;
};

struct State {
  TT X, Y, Z, T;
  BlockTT W;
  bool has_W = false;
  BlockTT EX, EZ, ET;                // warm starts of the step-length eigenvectors
  bool has_EX = false, has_EZ = false;
  BlockTT EXc, EZc;                  // warm starts of the positive-definiteness checks
  bool has_EXc = false, has_EZc = false;
  TT dX, dY, dZ, dT;                 // last Newton direction (corrector)
  double eta = 1e-3;
  int iter = 0;
  bool frame_capped = false;         // a Newton frame has reached the rank cap: enrichment is off
  std::vector<double> psi_hist;      // residual measures of the last accepted iterates (windowed control)
  bool finishing = false;            // in the finishing phase (PD barrier relaxation, merit acceptance)
  double nu = 0.0;                   // current relaxation M + nu I >= 0 of the finishing phase
  unsigned long long seed = 12345;
};

Problem build_problem(int kind, const TT& graph, const TT* negdeg, Ctx& c);
// The tensorised SDP given directly (Sec. 3.2): C, B_eq (and B_ineq) vec_TT
// vectors, the operators on vec_TT; Aineq == nullptr: no inequalities.
struct GenericSdp {
  const TT *C = nullptr, *Aeq = nullptr, *AeqT = nullptr, *Beq = nullptr, *KY = nullptr;
  const TT *Aineq = nullptr, *AineqT = nullptr, *Bineq = nullptr, *KT = nullptr;
  double sense = 1.0, q = 0.0, lam0 = 1.0, x0_ineq = 0.0, t0_ineq = 1e-3;
};
Problem build_problem_generic(const GenericSdp& g, Ctx& c);
void init_state(const Problem& P, const ttipm_params& prm, State& S, Ctx& c);
// One IPM iteration; fills info (measures at entry + the step taken).
// entry (optional): the measures of the current iterate, already computed by
// ipm_measures (the solve loop's stopping test), so that the step does not
// evaluate them again.
void ipm_step(const Problem& P, State& S, const ttipm_params& prm, ttipm_step_info& info, Ctx& c,
              const ttipm_step_info* entry = nullptr);
// Measures of the current iterate (mu, objectives, relative errors, gap).
void ipm_measures(const Problem& P, const State& S, ttipm_step_info& info, Ctx& c);
// The relative stopping criteria rel_gap <= stop_gap, eps_p, eps_d <= 2 stop_gap,
// and the absolute ones of the finishing phase ||R_p||, ||R_d||, <X, Z> < finish_abs.
bool ipm_relative_done(const ttipm_step_info& m, const ttipm_params& prm);
bool ipm_absolute_done(const ttipm_step_info& m, const ttipm_params& prm);

// Smallest generalised eigenvalue of (dM, M) over TT vectors of the given rank
// (two-site DMRG with Cholesky reduction of the projected pencil and `kick`
// random kick ranks per split; Sec. 3.4).
// Throws TT_ERR_NOT_PD if a projected M is not positive definite.
double min_gen_eig(const TT& M, const TT& dM, BlockTT& E, bool& have_E, int rank, int sweeps, int kick,
                   unsigned long long seed, Ctx& c);
// Largest alpha in (0, 1] with M + alpha dM psd, scaled by tau (Sec. 3.4).
double step_length(const TT& M, const TT& dM, BlockTT& E, bool& have_E, const ttipm_params& prm,
                   unsigned long long seed, Ctx& c);

}  // namespace ttipm
