// The learned block preconditioner: a two-hidden-layer ReLU network (FP32)
// that maps the features of a diagonal block (a, b) of a local system to a
// correction of its block-Jacobi inverse, M_b = B_b^{-1} + C_b / s_b, with
// hand-written forward, backward and Adam kernels.  The training data are
// probe pairs of the local systems the solver itself emits: for a probe x of
// the whole system and y = K x, the block residual r_b = x_b - B_b^{-1} y_b;
// the loss is the mean of w || r_b - C_b y_b / s_b ||^2, the block part of
// || x - M K x ||^2.
#pragma once

#include <vector>

#include "krylov.hpp"

namespace ttipm {

// device float buffer on the pool allocator
class FBuf {
 public:
  FBuf() = default;
  explicit FBuf(size_t n) { reserve(n); }
  void reserve(size_t n) { d_.reserve((n + 1) / 2); n_ = n > n_ ? n : n_; }
  float* get() const { return reinterpret_cast<float*>(d_.get()); }
  size_t size() const { return n_; }

 private:
  DevBuf d_;
  size_t n_ = 0;
};

struct MlpBatch {
  int N = 0, P = 0, n = 0;   // blocks, probes per block, block size
  const float* F = nullptr;  // [N][in]
  const float* R = nullptr;  // [N][P][n]
  const float* Y = nullptr;  // [N][P][n]
  const float* S = nullptr;  // [N]
  const float* W = nullptr;  // [N][P]
};

struct Mlp {
  int in = 0, H = 0, out = 0;
  long nparams = 0;
  FBuf params, grad, adam_m, adam_v;
  long adam_t = 0;
  // growable dataset of emitted local-system blocks (device)
  int ds_P = 0, ds_n = 0;
  long ds_N = 0, ds_cap = 0;
  FBuf dsF, dsR, dsY, dsS, dsW;
  // scratch
  FBuf z1, h1, z2, h2, o, dout, dh;

  void init(int in_, int H_, int out_, unsigned long long seed, Ctx& c);
  float* W1() const { return params.get(); }
  float* b1() const { return W1() + (long)H * in; }
  float* W2() const { return b1() + H; }
  float* b2() const { return W2() + (long)H * H; }
  float* W3() const { return b2() + H; }
  float* b3() const { return W3() + (long)out * H; }
  // out[N][out] = network(F[N][in])
  void forward(const float* F, int N, float* outp, Ctx& c);
  // loss of a batch (host double) and gradient into grad (device)
  double loss_grad(const MlpBatch& b, Ctx& c);
  void adam_step(float lr, Ctx& c);
  // append blocks to the dataset (device pointers, same layout as MlpBatch)
  void append(const MlpBatch& b, long cap, Ctx& c);
};

// Adam on shuffled mini-batches of data (device); hist[epoch] = mean batch loss.
void mlp_train(Mlp& net, const MlpBatch& data, int epochs, int batch, float lr, unsigned long long seed,
               std::vector<double>& hist, Ctx& c);

// Features and probe data of the (a, b) blocks of a local operator: F [nb][n*n+5]
// (normalised block entries, log10 of the block norm, 4 context scalars), S [nb] (block norms), and for
// nprobe seeded probes x: R = x_b - B_b^{-1} y_b, Y = y_b (y = K x) [nb][P][n].
// `apply_K` computes y = K x on [L][r][m][s] vectors.
void mlp_block_data(const BlockJacobi& raw, const BlockJacobi& inv, const std::function<void(const double*, double*)>& apply_K,
                    const float ctx[4], int nprobe, unsigned long long seed, FBuf& F, FBuf& R, FBuf& Y, FBuf& S,
                    FBuf& W, Ctx& c);
// inv.blk += C_b / s_b with C_b = network(features of raw) (the MLP preconditioner)
void mlp_correct_blocks(Mlp& net, const BlockJacobi& raw, BlockJacobi& inv, const float ctx[4], Ctx& c);

}  // namespace ttipm

// the opaque handle of the C ABI
struct tt_mlp {
  ttipm::Mlp net;
};
