/*
 * ttipm.h — C ABI of the MI355X tensor-train interior-point library.
 *
 * The library solves the semidefinite programs of the paper "An Inexact
 * Tensor-Train Primal-Dual Interior-Point Method for Semidefinite Programs"
 * (arXiv 2509.11890) with every matrix (X, Y, T, Z, the Newton direction and
 * the constraint operators) held in tensor-train (TT) form over d binary
 * modes, n = 2^d.  The primal SDP is Sec. 2.2, Def. "SDP"; its dual is
 * Def. "The Dual SDP"; the tensorised problem, vec_TT and the TT operators
 * are Sec. 3.1-3.3.
 *
 * Conventions used by every call
 *   - Storage: FP64, row-major, device memory.  A TT vector core k is
 *     [r_k][m][r_{k+1}]; a TT matrix (operator) core k is
 *     [R_k][m_out][m_in][R_{k+1}] (Def. "TT Matrix").  Index order is
 *     big-endian (core 0 holds the most significant digit) and the 2x2 mode
 *     of an n x n matrix is vectorised row-major, i = 2 alpha_k + beta_k,
 *     exactly as in the worked example of Def. "TT Vectorisation".
 *   - Ownership: every device pointer passed in is owned by the caller and
 *     must stay valid until the stream has finished the call.  Handles
 *     (ttipm_problem, ttipm_state) are owned by the library and released by
 *     their *_destroy call.  Handles are not thread-safe.
 *   - Streams: every call that launches work takes a hipStream_t (passed as
 *     void*, NULL = default stream) and is ordered on it.  Calls whose result
 *     decides a rank or a convergence test synchronise that stream; this is
 *     stated per call.
 *   - Errors: every call returns a status code (TT_OK = 0).  On failure
 *     tt_last_error() returns a thread-local message.  No C++ exception
 *     crosses this boundary.  A call that fails leaves its outputs undefined.
 */
#ifndef TTIPM_H
#define TTIPM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define TTIPM_API __attribute__((visibility("default")))
#else
#define TTIPM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
  TT_OK = 0,
  TT_ERR_ARG = 1,           /* invalid argument (shape, rank, pointer)          */
  TT_ERR_HIP = 2,           /* a HIP runtime call failed                        */
  TT_ERR_ALLOC = 3,         /* device allocation failed                         */
  TT_ERR_RANK_CAP = 4,      /* warning: a result was truncated at the rank cap  */
  TT_ERR_NOT_CONVERGED = 5, /* iteration limit reached                          */
  TT_ERR_NOT_PD = 6,        /* an iterate lost positive definiteness            */
  TT_ERR_NUMERIC = 7,       /* NaN or Inf detected                              */
  TT_ERR_BREAKDOWN = 8      /* Krylov breakdown                                 */
};

enum { TT_LEFT = 0, TT_RIGHT = 1 };
enum { TT_TOL_ABS = 0, TT_TOL_REL = 1 };

/* Text of the last error on this thread ("" if none). */
TTIPM_API const char* tt_last_error(void);

/* Library version string. */
TTIPM_API const char* tt_version(void);

/* sizeof of the caller-visible structs, in this order: tt_view, tt_proj_op,
   tt_local_block, tt_local_op, tt_solve_params, tt_solve_info,
   ttipm_problem_desc, tt_mlp_batch, tt_kernel_stat, ttipm_params,
   ttipm_step_info, ttipm_result.  Writes min(n, 12) values to out (host
   memory) and returns how many there are (12); a binding compares them with
   its own mirrors of the structs before any call.  Needs no GPU. */
TTIPM_API int tt_abi_sizes(size_t* out, int32_t n);

/* ---- TT views ----------------------------------------------------------- */
enum { TT_F64 = 0, TT_F32 = 1, TT_BF16 = 2 };

/*
 * A TT vector (m_in == 1) or TT matrix (m_in > 1) with d cores.
 *   ranks : host array of d+1 ranks, ranks[0] = ranks[d] = 1.  Calls that
 *           change ranks (tt_round) write the new ranks here.
 *   m_out : mode size of every core (4 for vec_TT vectors and operators,
 *           2 for TT matrices and plain vectors over binary modes).
 *   m_in  : 1 for a TT vector, the input mode size for an operator.
 *   cores : host array of d device pointers; core k holds
 *           ranks[k] * m_out * m_in * ranks[k+1] elements of dtype.
 *   capacity_rank : 0, or the largest rank every core buffer has room for
 *           (core k holds capacity ranks on both bonds); a call that writes
 *           a TT of data-dependent rank into the view never exceeds it.
 *   dtype : element type of the cores.  Every call of this header reads and
 *           writes TT_F64 views and rejects the others with TT_ERR_ARG; the
 *           field lets low-precision copies cross the boundary tagged.
 * A view with d = 0 is an absent argument where a call allows one.
 */
typedef struct {
  int32_t d;
  int32_t m_out;
  int32_t m_in;
  int32_t* ranks;
  double** cores;
  int32_t capacity_rank;
  int32_t dtype;
} tt_view;

/* ---- environments (interfaces) ------------------------------------------ */
/*
 * One step of the left or right environment recursion (Def. "Interface
 * Matrix"; the cached environments of the matrix-free local products in
 * Sec. 3.3).  With test TT V, operator O (NULL = identity) and trial TT U:
 *   dir = TT_LEFT : phi_out[a2][beta][c2] =
 *        sum V_k[a][i][a2] phi_in[a][alpha][c] O_k[alpha][i][j][beta] U_k[c][j][c2]
 *        phi_in is the environment of cores < k, phi_out that of cores <= k.
 *   dir = TT_RIGHT: phi_out[a][alpha][c] =
 *        sum V_k[a][i][a2] O_k[alpha][i][j][beta] U_k[c][j][c2] phi_in[a2][beta][c2]
 *        phi_in is the environment of cores > k, phi_out that of cores >= k.
 * For O == NULL the middle (operator-rank) index has size 1 and V, U must
 * have equal mode sizes.  V and U are TT vectors (m_in == 1); O has modes
 * V.m_out x U.m_out.  No synchronisation.
 */
TTIPM_API int tt_contract_interfaces(const tt_view* test, const tt_view* op, const tt_view* trial,
                           int32_t k, int32_t dir, const double* phi_in, double* phi_out,
                           void* stream);

/*
 * <Oi vi, Oj vj> for TT vectors vi, vj (m_in = 1, equal mode sizes) and
 * operators Oi, Oj on them (NULL = identity), without forming the images:
 * one left-to-right sweep over a four-layer environment
 * E[a][alpha][beta][c] (ranks of vi, Oi, Oj, vj), four GEMM stages per core.
 * The norm of a sum of operator images (a global residual K dU + R of the
 * Newton system, Sec. 3.3, Lemma "AMEn Directions as Inexact Newton
 * Directions") is a sum of such terms.  Device memory: the environment and two
 * stage buffers of max_k ranks(vi) ranks(Oi) ranks(Oj) ranks(vj) * m doubles.
 * Writes the value to *out (host).  Synchronises the stream.
 */
TTIPM_API int tt_op_inner(const tt_view* vi, const tt_view* Oi, const tt_view* vj, const tt_view* Oj, double* out,
                          void* stream);

/* ---- projected local operator -------------------------------------------- */
/*
 * A projected operator W^T O W at core k, applied matrix-free (Sec. 3.3):
 *   y[a][i][b] = sum phiL[a][alpha][a'] O_k[alpha][i][j][beta] x[a'][j][b'] phiR[b][beta][b']
 * core == NULL is the identity operator (R = Rp = 1, m_out = m_in).
 */
typedef struct {
  const double* phiL;   /* [r][R][r]   device */
  const double* core;   /* [R][m][m][Rp] device, or NULL */
  const double* phiR;   /* [rp][Rp][rp] device */
  int32_t R, Rp;
} tt_proj_op;

/*
 * One block of the local block system: y_row += coeff * P(op[nchain-1]) ... P(op[0]) x_col.
 * nchain = 2 expresses the chained products such as L_X^ Aeq^T^ of the
 * reduced projected system, eq. (reduced_kkt_system): the product of two
 * projected operators, never the projection of their product.
 */
typedef struct {
  int32_t row, col;
  double coeff;
  int32_t nchain;
  tt_proj_op op[2];
} tt_local_block;

/*
 * The local system at one core: L components, each a local core
 * [r][m][rp] (vectors x and y are [L][r][m][rp], component-major).
 */
typedef struct {
  int32_t r, rp, m, L;
  int32_t nblocks;
  const tt_local_block* blocks;   /* host array of nblocks */
  int32_t precision;              /* TTIPM_F64: FP64 MFMA contractions; TTIPM_MIXED: BF16
                                     operands with FP32 accumulation (vectors stay FP64) */
} tt_local_op;

/* y = K x in the precision of K->precision.  No synchronisation: the work is
 * enqueued on the stream (scratch is owned by the per-stream context). */
TTIPM_API int tt_local_matvec(const tt_local_op* K, const double* x, double* y, void* stream);

/*
 * y = K x exactly as tt_local_matvec (same kernels, same results), for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Every intermediate (the
 * permuted operator cores, chain buffers, the three GEMM stages' buffers and
 * the split-K partial sums) lives in one static device array of 64 MiB per
 * GPU, held from the first call on that GPU until the process ends; the call
 * never allocates or frees memory.  The caller still owns x and y.  The device
 * of the call is the current device; the stream must belong to it.  If the
 * call would need more than the 64 MiB (for one operator block about
 * r = 64, R = 128), it returns TT_ERR_ARG with the required size in
 * tt_last_error() and launches nothing.  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other threads) race and must
 * be serialised by the caller.  No synchronisation.
 */
TTIPM_API int tt_local_matvec_noalloc(const tt_local_op* K, const double* x, double* y, void* stream);

/* DIRECT: blocked LU with partial pivoting of the assembled dense K.
 * CHOLESKY: blocked Cholesky of the symmetric part of the assembled K, for
 * symmetric positive definite local operators; TT_ERR_NUMERIC if a pivot is
 * not positive. */
enum { TT_SOLVE_AUTO = 0, TT_SOLVE_DIRECT = 1, TT_SOLVE_GMRES = 2, TT_SOLVE_CHOLESKY = 3 };
enum { TT_PREC_NONE = 0, TT_PREC_BJACOBI = 1, TT_PREC_MLP = 2 };

typedef struct {
  int32_t method;       /* TT_SOLVE_*; AUTO = direct when L*r*m*rp <= direct_max */
  int32_t direct_max;   /* size limit of the dense direct solve (AUTO)             */
  int32_t restart;      /* GMRES restart length                                    */
  int32_t maxit;        /* GMRES iteration limit                                   */
  double rtol;          /* relative residual target ||b - K x|| <= rtol ||b||      */
  int32_t precond;      /* TT_PREC_*                                               */
  int32_t precision;    /* TTIPM_F64 or TTIPM_MIXED (see below)                    */
  const void* mlp;      /* tt_mlp handle when precond == TT_PREC_MLP               */
  float context[4];     /* context features of the MLP preconditioner (see tt_mlp) */
} tt_solve_params;

typedef struct {
  int32_t iters;        /* Krylov iterations (0 for the direct solve)            */
  int32_t method_used;  /* TT_SOLVE_DIRECT, TT_SOLVE_GMRES or TT_SOLVE_CHOLESKY  */
  int32_t precond_used; /* TT_PREC_* actually used (after the fallback rule)     */
  double rel_res;       /* true relative residual ||b - K x|| / ||b|| (FP64)      */
} tt_solve_info;

/*
 * Solve K x = rhs for the local system (Sec. 3.3: matrix-free GMRES on the
 * reduced projected system, or a dense direct solve when it is small).
 * With p->precision == TTIPM_MIXED the Arnoldi products use BF16-operand
 * contractions and every restart recomputes the true residual rhs - K x in
 * FP64 (GMRES as the inner solver of an iterative refinement), so rel_res is
 * an FP64 residual.  The direct methods always run in FP64.
 * p->precond: TT_PREC_BJACOBI applies the inverse of the (a, b) diagonal
 * blocks of K (L*m x L*m each) as a right preconditioner.
 * x holds the initial guess on entry and the solution on exit (x must not
 * alias rhs).  Synchronises
 * the stream (convergence tests).  Returns TT_ERR_NOT_CONVERGED if rtol was
 * not met within maxit (x then holds the best iterate).
 */
TTIPM_API int tt_local_solve(const tt_local_op* K, const double* rhs, double* x, const tt_solve_params* p,
                   tt_solve_info* info, void* stream);

/* ---- TT rounding ---------------------------------------------------------- */
/*
 * In-place TT rounding (Sec. 2.3, round_TT; the QR + truncated-SVD method of
 * Oseledets 2011): right-to-left Householder QR, then left-to-right truncated
 * SVD with per-bond budget eps / sqrt(d-1), eps = tol (TT_TOL_ABS) or
 * tol * ||t||_F (TT_TOL_REL), ranks capped at max_rank.  Ranks never grow, so
 * the caller's core buffers are reused; t->ranks is updated.  zeta_out (may be
 * NULL) receives ||t - round(t)||_F accumulated from the discarded singular
 * values (the spectral-shift size of Cor. 1).
 * ws: NULL = scratch from the library's caching device pool; else a
 * caller-owned, 256-byte aligned device region of ws_bytes from which every
 * device buffer of the call is taken (at least tt_round_workspace bytes; a
 * call that would need more returns TT_ERR_ARG with t unchanged).  Pinned host
 * staging of the norms stays library-owned.  Synchronises the stream.
 * Returns TT_ERR_RANK_CAP (a warning, result valid) if the cap truncated more
 * than the tolerance allowed.
 */
TTIPM_API int tt_round(tt_view* t, double tol, int32_t tol_mode, int32_t max_rank, double* zeta_out, void* ws,
                       size_t ws_bytes, void* stream);

/* Workspace bytes that always suffice for tt_round of t (any tolerance, any
 * cap): written to *bytes.  No device work. */
TTIPM_API int tt_round_workspace(const tt_view* t, size_t* bytes);

/* ---- the interior-point method --------------------------------------------- */
typedef struct ttipm_problem ttipm_problem;
typedef struct ttipm_state ttipm_state;

enum { TTIPM_MAXCUT = 0, TTIPM_THETA = 1, TTIPM_CC = 2, TTIPM_GENERIC = 3 };
enum { TTIPM_F64 = 0, TTIPM_MIXED = 1 };
enum { TTIPM_DIR_XZ = 0, TTIPM_DIR_AHO = 1 };

/*
 * Problem description.
 * Kinds built from a graph (Sec. 4): graph is a TT matrix with 2 x 2 modes,
 *   TTIPM_MAXCUT: the weighted adjacency A_G (Sec. 4.1);
 *   TTIPM_THETA : the 0/1 adjacency A_G (Sec. 4.2);
 *   TTIPM_CC    : the signed weights W = C+ - C-, zero diagonal (Sec. 4.3),
 *                 with negdeg the TT vector (m_out = 2) of C- 1;
 * the library builds C, A_eq, B_eq, K_Y (and A_ineq, K_T) itself.
 * TTIPM_GENERIC: the tensorised SDP of Sec. 3.2 given directly (Def. "SDP",
 * Def. "The Dual SDP" in TT form): maximise <C, X> subject to
 * A_eq vec_TT X = B_eq, A_ineq vec_TT X <= B_ineq (>= with ineq_sense = -1),
 * X psd.  C, B_eq, B_ineq are vec_TT vectors (m_out 4, m_in 1); A_eq, A_eq^T,
 * K_Y, A_ineq, A_ineq^T, K_T are operators on vec_TT (m_out = m_in = 4).  The
 * multipliers Y and T are padded to n x n (Sec. 3.2): K_Y and K_T are the
 * diagonal masks of their idle entries, and the active inequality mask 1_T is
 * taken as vec_TT(J) - K_T vec_TT(J).  Aineq.d = 0 means no inequalities.
 * q counts the inequality multipliers in mu = (<X,Z> + <T, s(X)>) / (n + q);
 * the initial point is X = lam0 I + x0_ineq A_ineq(J), Z = lam0 I, Y = 0,
 * T = t0_ineq A_ineq(J) (Sec. 5.1).  The graph kinds ignore these fields.
 * Every input is copied at create time; the caller's buffers may be freed
 * after the call.  All views are TT_F64.
 */
typedef struct {
  int32_t kind;
  tt_view graph;
  tt_view negdeg;   /* TTIPM_CC only (d = 0 otherwise) */
  tt_view C, Aeq, AeqT, Beq, KY;          /* TTIPM_GENERIC */
  tt_view Aineq, AineqT, Bineq, KT;       /* TTIPM_GENERIC with inequalities */
  int32_t ineq_sense;                     /* +1: A_ineq vec X <= B_ineq; -1: >= */
  double q;
  double lam0, x0_ineq, t0_ineq;
} ttipm_problem_desc;

TTIPM_API int ttipm_problem_create(const ttipm_problem_desc* desc, ttipm_problem** out);
TTIPM_API void ttipm_problem_destroy(ttipm_problem* p);

/* ---- learned block preconditioner ---------------------------------------- */
/*
 * A two-hidden-layer ReLU network (FP32) predicting, for each diagonal block
 * (a, b) of a local system (n = L*m unknowns per block), a correction C_b of
 * the block-Jacobi inverse: M_b = B_b^{-1} + C_b / s_b, s_b = ||B_b||_F.  Its
 * input is the block normalised by s_b (n*n values, row-major), log10(s_b)
 * and four context scalars (the IPM passes log10(mu), k/d, r/64, s/64), so
 * in_dim = n*n + 5 and out_dim = n*n.  The output layer starts at zero: an
 * untrained network is exactly the block-Jacobi preconditioner.
 * Training data are probe pairs of local systems: for a seeded Gaussian probe
 * x of the whole system and y = K x, the block residual r_b = x_b - B_b^{-1} y_b
 * and y_b; the loss is (1/N) sum_blocks sum_p w_p || r_b - C_b y_b / s_b ||^2
 * with w_p = (number of blocks) / ||x||^2, the block part of ||x - M K x||^2.
 * Parameters are flat FP32 in the order W1 [h][in], b1 [h], W2 [h][h], b2 [h],
 * W3 [out][h], b3 [out].  Handles are not thread-safe.
 */
typedef struct tt_mlp tt_mlp;

typedef struct {
  int32_t N, P, n;      /* blocks, probes per block, unknowns per block             */
  const float* F;       /* [N][n*n + 5] features (device)                           */
  const float* R;       /* [N][P][n] block-Jacobi residuals (device)                */
  const float* Y;       /* [N][P][n] probe images y_b (device)                      */
  const float* S;       /* [N] block norms (device)                                 */
  const float* W;       /* [N][P] probe weights (device)                            */
} tt_mlp_batch;

TTIPM_API int tt_mlp_create(int32_t in_dim, int32_t hidden, int32_t out_dim, int32_t seed, tt_mlp** out);
TTIPM_API void tt_mlp_destroy(tt_mlp* m);
TTIPM_API int64_t tt_mlp_num_params(const tt_mlp* m);
/* host copies of the flat parameter vector (count must equal tt_mlp_num_params) */
TTIPM_API int tt_mlp_get_params(const tt_mlp* m, float* host, int64_t count);
TTIPM_API int tt_mlp_set_params(tt_mlp* m, const float* host, int64_t count);
/* loss of a batch and its gradient (host, flat, num_params floats; may be NULL) */
TTIPM_API int tt_mlp_loss_grad(tt_mlp* m, const tt_mlp_batch* b, double* loss, float* grad_host, void* stream);
/* Append the blocks of local system K to the handle's dataset (at most cap
 * blocks in total): features with the given context, nprobe seeded probes. */
TTIPM_API int tt_mlp_collect(tt_mlp* m, const tt_local_op* K, const float* context, int32_t nprobe, int32_t seed,
                             int64_t cap, void* stream);
TTIPM_API int tt_mlp_dataset_size(const tt_mlp* m, int64_t* n_blocks);
/* Adam on shuffled mini-batches of data (NULL = the collected dataset);
 * loss_hist (host, epochs doubles, may be NULL) receives the mean loss per epoch. */
TTIPM_API int tt_mlp_train(tt_mlp* m, const tt_mlp_batch* data, int32_t epochs, int32_t batch, float lr, int32_t seed,
                           double* loss_hist, void* stream);
/* loss of data (NULL = the collected dataset) without updating the network */
TTIPM_API int tt_mlp_eval(tt_mlp* m, const tt_mlp_batch* data, double* loss, void* stream);

/* Kernel timing.  While profiling is on, every period-th launch of the
 * instrumented kernels (the FP64 and BF16 MFMA GEMMs, the Jacobi SVD, the LU
 * panel, the Lanczos eigen-solver of the step length, and the single-workgroup
 * Cholesky / LU / triangular solves as one group) is bracketed by HIP events
 * recorded on its launch stream.
 * tt_profile_stop synchronises on those events, turns profiling off and writes
 * up to cap records (one per instrumented kernel) into out; *count receives
 * the number of instrumented kernels.  flops and bytes are the algorithmic
 * counts of the timed launches (GEMM: 2 M N K flops; operands and result read
 * or written once), so flops / time is the achieved rate of those launches.
 * Profiling is process-wide and not meant to overlap with another profiled run. */
typedef struct {
  char name[48];
  int64_t launches;     /* launches while profiling was on                        */
  int64_t timed;        /* launches bracketed by events                           */
  double time_ms;       /* summed event time of the timed launches                */
  double flops;         /* algorithmic flops of the timed launches                */
  double bytes;         /* algorithmic bytes of the timed launches                */
} tt_kernel_stat;

TTIPM_API int tt_profile_start(int32_t period);
TTIPM_API int tt_profile_stop(tt_kernel_stat* out, int32_t cap, int32_t* count);

/* Parameters (defaults from ttipm_params_default follow Sec. 3.5 and Sec. 5.1). */
typedef struct {
  double eps_gap;       /* time-to-gap mark: rel_gap <= eps_gap, eps_p, eps_d <= 2 eps_gap */
  double stop_gap;      /* stop when rel_gap <= stop_gap and eps_p, eps_d <= 2 stop_gap   */
  double eta0;          /* initial forcing term (1e-3)                                    */
  double delta;         /* forcing-term floor (1e-4 in the paper)                         */
  double cmu;           /* eta <- max(min(eta, cmu mu), delta), cmu = 2                    */
  double tau;           /* fraction of the maximal step (reading: 0.95)                   */
  int32_t n_xz;         /* XZ warm-up iterations (3)                                      */
  int32_t max_iter;     /* IPM iteration limit                                            */
  int32_t rank_cap;     /* cap on the Newton-direction (frame) ranks                      */
  int32_t iter_rank_cap;/* cap on iterate ranks after rounding                            */
  int32_t amen_sweeps;  /* maximal AMEn half-sweeps per Newton solve                      */
  int32_t direct_max;   /* local systems up to this size are solved densely               */
  int32_t gmres_restart;
  int32_t gmres_maxit;
  int32_t precision;    /* TTIPM_F64 or TTIPM_MIXED                                       */
  int32_t precond;      /* TT_PREC_*                                                      */
  const void* mlp;      /* tt_mlp handle for TT_PREC_MLP (and the collect_probes dataset)  */
  int32_t eig_rank;     /* rank of the TT eigenvector in the step-length solver          */
  int32_t eig_sweeps;   /* ALS sweeps of the step-length solver                           */
  int32_t verbose;      /* print one line per iteration to stderr                          */
  int32_t kick;         /* enrichment directions per AMEn core move (2)                   */
  int32_t seed;         /* seed of the enrichment and step-length start vectors            */
  int32_t kick_sweeps;  /* enrichment only in the first kick_sweeps half-sweeps of a solve */
  int32_t collect_probes; /* > 0 and mlp set: every local system of the AMEn solves adds its
                           blocks with this many probes to the mlp handle's dataset        */
  int64_t collect_cap;  /* dataset size limit (blocks) for collect_probes                 */
  int32_t xz_fallback;  /* 1: redo an AHO iteration with the XZ direction when its predictor
                           solve ends at the rank cap above its residual target, or admits a
                           step below 1e-3 (Sec. 3.5); not with inequalities (0)            */
  int32_t eig_kick;     /* random kick ranks per core split of the step-length DMRG (2)   */
  int32_t g4_window;    /* M of the windowed residual control (Sec. 3.3, (G4)): once the XZ
                           warm-up is over, an update whose residual measure
                           Psi = ||R_p|| + ||R_d|| + mu exceeds the largest Psi of the last
                           M + 1 iterates by more than the rounding budget is damped (both
                           step lengths halved) and retried; 0 = off (4)                 */
  int32_t g4_retries;   /* damped retries of the windowed control per iteration (3); after
                           the last one the trial with the smallest Psi is taken          */
  int32_t shift_mode;   /* Cor. 1 shift of the rounded X, Z, T: 1 = the whole rounding error
                           zeta (keeps positive definiteness also when iter_rank_cap forces
                           a larger truncation than the tolerance; default), 0 = only the
                           part within the tolerance budget                               */
  int32_t newton_check; /* 1: evaluate the global FP64 residual ||K dU + R|| / ||R|| of each
                           corrector direction (ttipm_step_info.newton_res); with
                           precision TTIPM_MIXED a direction above eta is then refined by
                           FP64 AMEn sweeps warm-started from it (1)                      */
  int32_t refine_sweeps;/* FP64 half-sweeps of one such refinement (2)                    */
  int32_t combine_multipliers; /* 1: with inequalities whose masks are disjoint
                           ((I - K_Y)(I - K_T) = 0), Y and T updates share one padded block
                           dL of the Newton system (Sec. 3.5, Combined Multiplier Storage):
                           two block rows and columns instead of three (1)               */
  int32_t amen_global_stop; /* 1: an AMEn solve whose frame the rank cap has truncated stops
                           after the half-sweep at which the global FP64 residual ratio
                           ||K dU + R|| / ||R|| meets eta or improves on the previous
                           half-sweep's by less than 10 % (evaluated after every half-sweep
                           of such a solve) (1)                                            */
  int32_t finish;       /* 1: finishing phase (Sec. 3.5, Relaxing the Positive Definiteness
                           Barrier): once the relative stopping criteria hold, ttipm_solve
                           goes on until ||R_p||_F, ||R_d||_F, <X, Z> < finish_abs; in that
                           phase the step lengths and the PD safeguard use M + nu I >= 0
                           and an update is accepted only if ||R_p|| + ||R_d|| + |<X, Z>|
                           decreases with eps_p, eps_d and rel_gap within max(current, the
                           relative bound); after damped retries a rejected iteration keeps
                           the iterate and raises nu (1e-7, then x10, at most
                           finish_nu_max).  The result meets the relative criteria (0)    */
  double finish_abs;    /* absolute targets of the finishing phase (1e-3)                 */
  double finish_nu_max; /* largest relaxation nu of the finishing phase (1e-3)            */
  int32_t enrich;       /* AMEn enrichment (Sec. 2.3): 1 = the leading directions of the
                           Newton residual K dU + R sketched with a seeded Gaussian TT on
                           the side ahead of the block (1); 0 = seeded random directions,
                           off once rank_cap truncates.  Both fill only capacity left
                           under rank_cap                                                 */
} ttipm_params;

TTIPM_API void ttipm_params_default(ttipm_params* p);

/* Initial point of Sec. 5.1: X = Z = lambda* I, Y = 0 (+ the inequality start). */
TTIPM_API int ttipm_state_create(const ttipm_problem* p, const ttipm_params* prm, ttipm_state** out);
TTIPM_API void ttipm_state_destroy(ttipm_state* s);

/* Per-iteration record. */
typedef struct {
  int32_t iter, direction, sweeps_pred, sweeps_corr, krylov_iters;
  int32_t rank_x, rank_y, rank_z, rank_w;
  double mu, pobj, dobj, rel_gap, eps_p, eps_d, eps_c;
  double norm_rp, norm_rd, xz;      /* ||R_p||_F, ||R_d||_F and <X, Z> (+ <T, slack>) of the entry iterate */
  double alpha_p, alpha_d, sigma, eta;
  double alpha_p_max, alpha_d_max;  /* Thm. 1 step bounds from the TT eigen-solver, before tau and
                                       the PD check (1e6 when the direction has no bound) */
  int32_t backtracks;               /* step halvings forced by the positive-definiteness check */
  int32_t mlp_used, mlp_fallbacks;  /* local solves with the MLP preconditioner kept / replaced by
                                       block Jacobi under the fallback rule */
  int32_t xz_fallback;              /* 1 when this iteration fell back from AHO to XZ */
  int32_t g4_retries;               /* damped retries of the windowed residual control */
  double psi;                       /* residual measure ||R_p|| + ||R_d|| + mu of the accepted update
                                       (of the entry iterate when the control is off) */
  double zeta_x, zeta_x_cap;        /* rounding error ||X - X~||_F of the accepted update and its
                                       part forced by iter_rank_cap (only the rest, within the
                                       tolerance budget, is added as the Cor. 1 shift) */
  double zeta_z, zeta_z_cap;        /* the same for Z */
  double newton_res;                /* ||K dU + R|| / ||R|| of the corrector direction, FP64, after any
                                       refinement (0 when newton_check is off; -1 when an operator-image
                                       environment of the check would exceed 256 MiB) */
  int32_t refine_sweeps;            /* FP64 refinement half-sweeps of the corrector (mixed precision) */
  double t_check;                   /* seconds spent on the residual check and refinement */
  int32_t finishing;                /* 1 in the finishing phase */
  int32_t finish_rejected;          /* 1 when the finishing phase kept the iterate (no acceptable step) */
  double nu;                        /* barrier relaxation nu of this iteration (finishing phase) */
  double t_env, t_solve, t_svd, t_step, t_round, t_total;  /* seconds, this iteration: host time
                                    between synchronisation points, so GPU work a phase queues without
                                    waiting for it (the end of a local solve or of a split, environment
                                    updates) is counted in the phase that next waits */
} ttipm_step_info;

/*
 * One IPM iteration (Alg. 1): residuals and mu, Mehrotra predictor and
 * corrector Newton solves by block AMEn, step lengths (Sec. 3.4), update and
 * rounding with spectral shift (Cor. 1), eta update (Sec. 3.5).  info
 * receives the measures of the iterate at entry and the step taken.
 * Synchronises the stream.
 */
TTIPM_API int ttipm_step(ttipm_problem* p, ttipm_state* s, const ttipm_params* prm, ttipm_step_info* info,
               void* stream);

typedef struct {
  int32_t status;       /* TT_OK: the relative criteria (stop_gap) hold; with the finishing
                           phase on, the solve went on from there until the absolute ones,
                           max_iter or a stall, and the result still meets the relative
                           ones.  TT_ERR_NOT_CONVERGED: max_iter or a stall (both step
                           lengths < 1e-3 in five consecutive iterations) before the
                           relative criteria; TT_ERR_NOT_PD: an iterate lost positive
                           definiteness.  The other fields describe the last accepted
                           iterate in every case. */
  int32_t iterations;
  double time_to_gap;   /* seconds to the eps_gap mark (-1 if not reached)          */
  double time_total;
  double pobj, dobj, rel_gap, eps_p, eps_d;
  double norm_rp, norm_rd, xz;  /* ||R_p||_F, ||R_d||_F, <X, Z> (+ <T, slack>) */
  int32_t finish_iterations;    /* iterations spent in the finishing phase */
  int32_t absolute_met;         /* 1 when ||R_p||_F, ||R_d||_F, <X, Z> < finish_abs */
} ttipm_result;

/*
 * Iterate ttipm_step until the stopping test, max_iter or a stall.  log (may
 * be NULL) receives up to log_cap per-iteration records.  Returns TT_OK with
 * res->status describing how the run ended.  Synchronises the stream.
 */
TTIPM_API int ttipm_solve(ttipm_problem* p, ttipm_state* s, const ttipm_params* prm, ttipm_result* res,
                ttipm_step_info* log, int32_t log_cap, void* stream);

/*
 * Copy one iterate to the host: which = 'X', 'Y', 'Z' or 'T' for the
 * iterates, 'x', 'y', 'z', 't' for the components of the last Newton
 * direction (the corrector of the last ttipm_step).  ranks_out
 * receives d+1 ranks; cores are packed one after another into host_out
 * (capacity cap doubles).  Returns TT_ERR_ARG if cap is too small (the
 * required size is written to *needed when needed != NULL).
 */
TTIPM_API int ttipm_state_export(const ttipm_state* s, int32_t which, int32_t* ranks_out, double* host_out,
                       size_t cap, size_t* needed);

/*
 * Replace one iterate ('X', 'Y', 'Z' or 'T') with a TT given on the host, in
 * the packing of ttipm_state_export (d+1 ranks, boundary ranks 1; cores one
 * after another, count doubles in all): checkpoint / resume of a solve.  The
 * warm starts of the Newton frame and of the step-length eigenvectors are
 * kept.  Returns TT_ERR_ARG on a rank or size mismatch.  Synchronises.
 */
TTIPM_API int ttipm_state_import(ttipm_state* s, int32_t which, const int32_t* ranks, const double* host_in,
                                 size_t count);

#ifdef __cplusplus
}
#endif
#endif /* TTIPM_H */
